// HIP kernels of the space-time BDF1 Newton iteration for gfx950.
//
//  k_residual      all levels at once: r^n = -(u^n - u^{n-1} + tau F(u^n)) (Eq. (5)
//                  right-hand side), the rows of A_n when requested, the per-level
//                  Gershgorin radius of D^{-1} A_n (which fixes the inner Chebyshev
//                  interval) and max |r|.
//  k_level_solve   one level of the block inverse of Eq. (7): b = r^n + du^{n-1}
//                  (the -I block of Eq. (6)), then A_n du^n = b by restarted
//                  Jacobi-preconditioned Chebyshev passes. Each work-group owns a
//                  tile and keeps a 64 x 64 region (tile + halo) in registers, so all
//                  sweeps of a launch run without leaving the chip: x-neighbours move
//                  between lanes by DPP, y-neighbours between waves through LDS. The
//                  halo is as deep as the number of neighbour exchanges of the launch,
//                  which makes the tile values identical to a global sweep.
//  k_update        U += dU at every level and per-block sums of dU^2 (the RMS update
//                  norm of Section 8.1), reduced in fixed order by k_reduce_sum.
#include "pts_device.hpp"
#include "pts_mg.hpp"

namespace pts {

// ------------------------------------------------------------------ residual
// Block of 64 x 4 threads sweeping kResRows rows of one level; grid.x = tiles of the
// level, grid.y = level. Per-level maxima of |r| and of the Gershgorin radius go to
// lvl_bits[2n] and lvl_bits[2n+1] (zeroed before the launch); k_level_max folds them.
// R and coef may be NULL.
constexpr int kResRows = 16;

template <int BC, int FORM>
__global__ __launch_bounds__(256) void k_residual(KProb p0, const double* __restrict__ U,
                                                  const double* __restrict__ u0,
                                                  double* __restrict__ R, double* __restrict__ coef,
                                                  unsigned long long* __restrict__ lvl_bits) {
  const int n = blockIdx.y;
  const KProb p = at_level(p0, n);
  const int tilesx = (p.nx + 63) >> 6;
  const int x = (blockIdx.x % tilesx) * 64 + (threadIdx.x & 63);
  const int y0 = (blockIdx.x / tilesx) * kResRows + (threadIdx.x >> 6);
  const size_t ns = (size_t)p.nx * p.ny;
  const double* un = U + (size_t)n * ns;
  const double* up = n == 0 ? u0 : U + (size_t)(n - 1) * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
  double rabs = 0.0, rho = 0.0;
#pragma unroll 1
  for (int y = y0; y < y0 + kResRows; y += 4) {
    if (x < p.nx && y < p.ny) {
      const Nb u = gather<BC>(p, un, bd, x, y);
      const size_t i = (size_t)y * p.nx + x;
      Row5 a;
      const double F = eval_point<BC, FORM>(p, u, x, y, a);
      const double r = -(u.P - up[i] + p.dt * F);
      if (R) R[(size_t)n * ns + i] = r;
      rabs = nanmax(rabs, fabs(r));
      rho = nanmax(rho, (FORM == kFormConstVisc ? gersh(a, p.ic0) : gersh(a)));
      if (coef) {
        double* c = coef + (size_t)n * 5 * ns + i;
        c[0] = a.C;
        c[ns] = a.W;
        c[2 * ns] = a.E;
        c[3 * ns] = a.S;
        c[4 * ns] = a.N;
      }
    }
  }
  __shared__ double red[2][4];
  rabs = wave_max(rabs);
  rho = wave_max(rho);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = rabs;
    red[1][w] = rho;
  }
  __syncthreads();
  if (threadIdx.x == 0 && lvl_bits) {
    atomic_max_nonneg(lvl_bits + 2 * n, nanmax(nanmax(red[0][0], red[0][1]), nanmax(red[0][2], red[0][3])));
    atomic_max_nonneg(lvl_bits + 2 * n + 1, nanmax(nanmax(red[1][0], red[1][1]), nanmax(red[1][2], red[1][3])));
  }
}

// out[0] = max_n lvl[2n] (max |r|), out[1] = max_n lvl[2n+1] (max radius); one block.
__global__ __launch_bounds__(256) void k_level_max(const unsigned long long* __restrict__ lvl, int nt,
                                                   unsigned long long* __restrict__ out) {
  unsigned long long a = 0, b = 0;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) {
    a = lvl[2 * i] > a ? lvl[2 * i] : a;
    b = lvl[2 * i + 1] > b ? lvl[2 * i + 1] : b;
  }
  __shared__ unsigned long long ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ra[threadIdx.x] = ra[threadIdx.x + o] > ra[threadIdx.x] ? ra[threadIdx.x + o] : ra[threadIdx.x];
      rb[threadIdx.x] = rb[threadIdx.x + o] > rb[threadIdx.x] ? rb[threadIdx.x + o] : rb[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ra[0];
    out[1] = rb[0];
  }
}

// -------------------------------------------------------------- level solve
// The register-resident region is 64 lanes (x) by kWaves waves of kRows rows (y).
constexpr int kRows = 4;
constexpr int kWaves = 16;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxSweeps = 64;  // longest Chebyshev pass one launch may run

// Exchange of the first and last row of every wave with the neighbouring waves via LDS.
// buf holds 2 parities x kWaves x {bottom row, top row} x 64 lanes.
template <typename T>
struct YNb {
  T s0, nM;  // south neighbour of row 0, north neighbour of row kRows-1
};

template <typename T>
__device__ __forceinline__ YNb<T> y_exchange(const T (&v)[kRows], T* buf, int& par, int wave, int lane) {
  T* b = buf + par * (kWaves * 2 * 64);
  b[(wave * 2 + 0) * 64 + lane] = v[0];
  b[(wave * 2 + 1) * 64 + lane] = v[kRows - 1];
  __syncthreads();
  YNb<T> r;
  r.s0 = wave > 0 ? b[((wave - 1) * 2 + 1) * 64 + lane] : T(0);
  r.nM = wave < kWaves - 1 ? b[((wave + 1) * 2 + 0) * 64 + lane] : T(0);
  par ^= 1;
  return r;
}

// Chebyshev weights for the Jacobi iteration matrix with spectral radius bound rho
// (Golub-Varga semi-iteration): omega_1 = 1, omega_2 = 1/(1 - rho^2/2),
// omega_{k+1} = 1/(1 - rho^2 omega_k / 4). One thread fills the table in LDS while the
// other threads load the region.
// Called by (at least) the first wave with the same rho in every lane: lane s writes
// omega_s = 2 T_{s-1}(1/rho) / (rho T_s(1/rho)) (omega_1 = 1), the closed form of the
// recurrence omega_{s+1} = 1 / (1 - rho^2 omega_s / 4), omega_2 = 2 / (2 - rho^2); each lane
// runs the three-term recurrence of the Chebyshev polynomials T to its own s, so the
// divisions are independent instead of a dependent chain. (rho >= 1e-3 keeps T_63(1/rho)
// below 1e210.)
__device__ __forceinline__ void cheb_table(double* om, double rho, int sweeps) {
  const int s = threadIdx.x;
  if (s < 1 || s > sweeps || s >= kMaxSweeps) return;
  if (s == 1) {
    om[1] = 1.0;
    return;
  }
  const double x = 1.0 / rho;
  double tp = 1.0, tc = x;  // T_{k-1}, T_k at k = 1
  for (int k = 1; k < s; ++k) {
    const double tn = 2.0 * x * tc - tp;
    tp = tc;
    tc = tn;
  }
  om[s] = 2.0 * tp / (rho * tc);
}

__device__ __forceinline__ double clamp_rho(double rho) { return fmin(fmax(rho, 1e-3), 0.999); }

// Register-resident state of one region of a level: Jacobi-scaled rows of A_n (T; the
// off-diagonals stored negated, so a sweep is a chain of fused multiply-adds from d), the
// FP64 rows (only for FP32 inner arithmetic), right-hand side b and iterate X.
template <typename T>
struct RegionSolve {
  static constexpr bool kF64 = sizeof(T) == sizeof(double);
  double cC[kRows], cW[kRows], cE[kRows], cS[kRows], cN[kRows];
  double bb[kRows], X[kRows];
  T nW[kRows], nE[kRows], nS[kRows], nN[kRows], iC[kRows];  // -W/C, -E/C, -S/C, -N/C and 1/C

  __device__ __forceinline__ void set_row(int k, const Row5& a) { set_row(k, a, 1.0 / a.C); }
  // The constant-viscosity form's Jacobi-scaled row straight from the host-folded coefficients
  // (one fused multiply-add per entry, no scaling pass); a (unscaled) feeds the FP64 rows of
  // the FP32 inner type.
  __device__ __forceinline__ void set_row_const_visc(int k, const KProb& p, const Nb& u, const Row5& a) {
    iC[k] = T(p.ic0);
    nW[k] = T(fma(p.bxs, u.W, p.axs));
    nE[k] = T(fma(-p.bxs, u.E, p.axs));
    nS[k] = T(fma(p.bys, u.S, p.ays));
    nN[k] = T(fma(-p.bys, u.N, p.ays));
    if (!kF64) {
      cC[k] = a.C;
      cW[k] = a.W;
      cE[k] = a.E;
      cS[k] = a.S;
      cN[k] = a.N;
    }
  }
  // inv = 1 / a.C given (known without a division for some forms)
  __device__ __forceinline__ void set_row(int k, const Row5& a, double inv) {
    iC[k] = T(inv);
    nW[k] = T(-a.W * inv);
    nE[k] = T(-a.E * inv);
    nS[k] = T(-a.S * inv);
    nN[k] = T(-a.N * inv);
    if (!kF64) {
      cC[k] = a.C;
      cW[k] = a.W;
      cE[k] = a.E;
      cS[k] = a.S;
      cN[k] = a.N;
    }
  }

  // `passes` restarted Chebyshev passes of `sweeps` sweeps on A X = b, each pass from the
  // FP64 residual of the current X (haveX = false: X = 0 and the first residual is b).
  // Neighbour exchanges: (sweeps - 1) per pass, plus one per pass that starts from X.
  __device__ void run(int passes, int sweeps, bool haveX, const double* om, double* lds, int wave, int lane) {
    int par = 0;
    T* ldst = reinterpret_cast<T*>(lds);
    for (int pass = 0; pass < passes; ++pass) {
      T d[kRows];
      if (haveX) {
        const YNb<double> yn = y_exchange<double>(X, lds, par, wave, lane);
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
          const double xs = k == 0 ? yn.s0 : X[k - 1];
          const double xn = k == kRows - 1 ? yn.nM : X[k + 1];
          const double xw = lane_from_left(X[k]);
          const double xe = lane_from_right(X[k]);
          if (kF64) {
            double t = fma(double(iC[k]), bb[k], -X[k]);
            t = fma(double(nW[k]), xw, t);
            t = fma(double(nE[k]), xe, t);
            t = fma(double(nS[k]), xs, t);
            d[k] = T(fma(double(nN[k]), xn, t));
          } else {
            const double ax = cC[k] * X[k] + cW[k] * xw + cE[k] * xe + cS[k] * xs + cN[k] * xn;
            d[k] = T((bb[k] - ax) / cC[k]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < kRows; ++k) d[k] = T(bb[k]) * iC[k];
      }
      // Chebyshev on D^{-1} A x = D^{-1} d from x_0 = 0, x_1 = D^{-1} d; with the scaled
      // rows, x_s = x_{s-2} + omega_s (d - x_{s-2} - offdiag(x_{s-1})). xa and xb hold the
      // two most recent iterates and are overwritten alternately.
      T xa[kRows], xb[kRows];
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        xa[k] = T(0);
        xb[k] = d[k];
      }
      int s = 2;
      for (; s + 1 <= sweeps; s += 2) {
        sweep(xa, xb, d, T(om[s]), ldst, par, wave, lane);
        sweep(xb, xa, d, T(om[s + 1]), ldst, par, wave, lane);
      }
      const bool odd = s <= sweeps;
      if (odd) sweep(xa, xb, d, T(om[s]), ldst, par, wave, lane);
#pragma unroll
      for (int k = 0; k < kRows; ++k) X[k] += double(odd ? xa[k] : xb[k]);
      haveX = true;
    }
  }

  // xold <- xold + w (d - offdiag(xcur) - xold): one Chebyshev step written over x_{s-2}.
  __device__ __forceinline__ void sweep(T (&xold)[kRows], const T (&xcur)[kRows], const T (&d)[kRows], T w,
                                        T* ldst, int& par, int wave, int lane) {
    const YNb<T> yn = y_exchange<T>(xcur, ldst, par, wave, lane);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const T xs = k == 0 ? yn.s0 : xcur[k - 1];
      const T xn = k == kRows - 1 ? yn.nM : xcur[k + 1];
      const T xw = lane_from_left(xcur[k]);
      const T xe = lane_from_right(xcur[k]);
      T t = fma(nW[k], xw, d[k]);
      t = fma(nE[k], xe, t);
      t = fma(nS[k], xs, t);
      t = fma(nN[k], xn, t);  // d - offdiag(xcur)
      xold[k] = fma(w, t - xold[k], xold[k]);
    }
  }
};

// Region node of (lane, row) in domain coordinates; returns false for a Dirichlet node
// outside the domain (inactive: zero row, zero data).
template <int BC>
__device__ __forceinline__ bool region_node(const KProb& p, int gx, int gy, int& x, int& y) {
  if (BC == 1) {
    // regions start at most kMaxHalo nodes before the domain and end at most 64 nodes
    // after a tile origin, so one conditional step wraps when the level is >= 64 wide
    if (p.nx >= 64 && p.ny >= 64) {
      x = gx < 0 ? gx + p.nx : (gx >= p.nx ? gx - p.nx : gx);
      y = gy < 0 ? gy + p.ny : (gy >= p.ny ? gy - p.ny : gy);
    } else {
      x = wrap(gx, p.nx);
      y = wrap(gy, p.ny);
    }
    return true;
  }
  x = gx;
  y = gy;
  return gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny;
}

__device__ __forceinline__ bool in_tile(const Geo& g, const KProb& p, int lane, int row, int gx, int gy) {
  const int lx = g.whole ? lane : lane - g.H;
  const int ly = g.whole ? row : row - g.H;
  return lx >= 0 && lx < g.TX && ly >= 0 && ly < g.TY && gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny;
}

// Bulk schedule, one launch per level (or per group of passes of a level):
// X = A_n^{-1}(rn + dUprev), rn the level's right-hand side (r^n for the block inverse of
// Eq. (7), or a Theorem-1 chain vector), dUprev (nullable) du^{n-1}. Xin (nullable) is the
// starting iterate from a previous launch; Xout receives the tile values. One work-group
// per tile of the level.
template <typename T, int BC>
__device__ __forceinline__ void level_solve_tile(const KProb& p, int n, int tile, const double* __restrict__ U,
                                                 const double* __restrict__ rn,
                                                 const double* __restrict__ dUprev,
                                                 const double* __restrict__ Xin, double* __restrict__ Xout,
                                                 const double* __restrict__ rho_lvl, const Geo& g, int passes,
                                                 int sweeps, double* lds_raw, double* om) {
  const int lane = threadIdx.x & 63;
  // wave index as a wave-uniform value: row indices, their products with the row stride and
  // the periodic wrap of rows are then scalar work
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = tile % g.tilesx, ty = tile / g.tilesx;
  const int rx0 = g.whole ? 0 : tx * g.TX - g.H;
  const int ry0 = g.whole ? 0 : ty * g.TY - g.H;
  const size_t ns = (size_t)p.nx * p.ny;
  const double* un = U + (size_t)n * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
  cheb_table(om, clamp_rho(rho_lvl[2 * n + 1]), sweeps);

  RegionSolve<T> rs;
  unsigned idx[kRows];
  const int gx = rx0 + lane;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    int x, y;
    const bool act = region_node<BC>(p, gx, ry0 + wave * kRows + k, x, y);
    idx[k] = act ? (unsigned)y * (unsigned)p.nx + x : ~0u;
    Row5 a;
    if (act) {
      Nb u = gather<BC>(p, un, bd, x, y);
      (void)eval_point<BC>(p, u, x, y, a);
      rs.bb[k] = ld(rn, idx[k]) + (dUprev ? ld(dUprev, idx[k]) : 0.0);
      rs.X[k] = Xin ? ld(Xin, idx[k]) : 0.0;
    } else {
      a.C = 1.0;
      a.W = a.E = a.S = a.N = 0.0;
      rs.bb[k] = 0.0;
      rs.X[k] = 0.0;
    }
    rs.set_row(k, a);
  }
  __syncthreads();  // omega table
  rs.run(passes, sweeps, Xin != nullptr, om, lds_raw, wave, lane);
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int row = wave * kRows + k;
    if (idx[k] != ~0u && in_tile(g, p, lane, row, gx, ry0 + row)) st(Xout, idx[k], rs.X[k]);
  }
}

template <typename T, int BC>
__global__ __launch_bounds__(kThreads) void k_level_solve(KProb p, int n, const double* __restrict__ U,
                                                          const double* __restrict__ rn,
                                                          const double* __restrict__ dUprev,
                                                          const double* __restrict__ Xin,
                                                          double* __restrict__ Xout,
                                                          const double* __restrict__ rho_lvl, Geo g,
                                                          int passes, int sweeps) {
  __shared__ double lds_raw[2 * kWaves * 2 * 64];
  __shared__ double om[kMaxSweeps];
  level_solve_tile<T, BC>(at_level(p, n), n, blockIdx.x, U, rn, dUprev, Xin, Xout, rho_lvl, g, passes, sweeps,
                          lds_raw, om);
}

// Batched bulk schedule: independent instances with their own sizes, level counts and
// inner plans. Launch (n, l) solves, for every instance that has level n and at least
// l + 1 launches in its plan, launch l of that level (packs[l] passes of its sweeps, the
// same ping-pong between its scratch level and du^n as the one-instance chain). Work items
// are (instance, tile) pairs sorted by level count, so the grid of level n is a prefix.
constexpr int kMaxPacks = 64;
struct BatchDesc {
  KProb p;
  Geo g;
  const double* U;
  const double* R;
  double* dU;
  double* Xs;
  const double* rho;
  int npacks;  // launches per level of this instance's plan (0: instance inactive)
  int sweeps;
  int packs[kMaxPacks];
};

template <typename T, int BC>
__global__ __launch_bounds__(kThreads) void k_level_solve_batched(const BatchDesc* __restrict__ descs,
                                                                  const int2* __restrict__ items, int n, int l) {
  __shared__ double lds_raw[2 * kWaves * 2 * 64];
  __shared__ double om[kMaxSweeps];
  const int2 it = items[blockIdx.x];
  const BatchDesc* d = descs + it.x;
  const int nl = d->npacks;
  if (n >= d->p.nt || l >= nl) return;  // uniform over the work-group
  const KProb p = at_level(d->p, n);
  const Geo g = d->g;
  const size_t ns = (size_t)p.nx * p.ny;
  double* out = d->dU + (size_t)n * ns;
  double* xo = ((nl - 1 - l) % 2 == 0) ? out : d->Xs;
  const double* xin = l == 0 ? nullptr : (((nl - l) % 2 == 0) ? out : d->Xs);
  const double* prev = n == 0 ? nullptr : d->dU + (size_t)(n - 1) * ns;
  level_solve_tile<T, BC>(p, n, it.y, d->U, d->R + (size_t)n * ns, prev, xin, xo, d->rho, g, d->packs[l], d->sweeps,
                          lds_raw, om);
}

// ---------------------------------------- multigrid-preconditioned level solves (Dirichlet heat)
// For stiff Dirichlet heat levels the block A_n = I + tau dF/du is solved by Chebyshev
// iteration preconditioned with M = I + tau mu_a (-Delta_h), the constant-coefficient
// five-point operator, whose inverse is approximated by one multigrid V-cycle (pts_mg.hpp).
// With mu in [mu_a, mu_hi] the spectrum of M^{-1} A lies near [1, mu_hi / mu_a] (times a
// margin for the non-symmetric mu' terms of the Jacobian); the V-cycle B has spec(B M) in
// [kMgLow, 1], which widens the interval's lower end.
// Iteration k of level n: r = b - A x in FP64 from U (k_pc_resid, float32 r), z = B r (the
// V-cycle launches), d = c0 d + c1 z, x += d (ChebStep, applied once, where the V-cycle writes
// its finest grid: k_mg_up, or k_mg_lds where the whole V-cycle runs in LDS).
constexpr int kMaxCheb = 48;  // Chebyshev iterations per level solve
constexpr int kStat = 6;      // words of a pipelined lane's statistics per level
// One level solver's arrays. In the bulk schedule there is one per instance (stage 0, full
// space-time R and dU). In the pipelined schedule there is one per (instance, Newton stage s),
// a "lane": a launch for diagonal D has lane s work on level n = D - s, with its residual in a
// level buffer (rmask 0) and its update in a ring of two levels (dmask 1).
struct PcDesc {
  KProb p;
  double* U;          // iterate [nt][N][N]
  double* R;          // residual: level n at R + (n & rmask) N^2
  double* dU;         // update: level n at dU + (n & dmask) N^2; the level solve iterates in it
                      // (bulk schedule; pipelined lanes iterate in the float32 ring dxf)
  float* r;           // [N][ld] level residual b - A x (float32)
  float* z;           // [N][ld] B r
  float* d;           // [N][N] Chebyshev direction (float32: the inner solve's precision)
  int* K;             // [nt] iterations of level n (the interval follows the level's max |u|)
  float2* c;          // [nt][kMaxCheb]: d_k = c.x d_{k-1} + c.y z_k (c.x = 0 at k = 0)
  int active;
  int ld;             // row stride of the float32 arrays (N)
  int stage;          // the lane's Newton stage s (0 in the bulk schedule)
  int rmask, dmask;   // -1 in the bulk schedule
  // pipelined schedule only
  int last;                // the lane after the last stage: update and residual, no level solve
  const double* u0;        // the initial condition (level -1)
  double* park_out;        // lane s-1's park: U^(s-1) of the level this lane updates
  const double* park_in;   // U^(s) of level n-1, parked by lane s+1 (NULL: read U)
  float* dxf;              // the lane's update ring (float32, two levels): the level solve's iterate
  const float* dprev;      // lane s-1's update ring
  unsigned long long* stat;  // [nt][kStat] max |U^(s)_n|, max |R^(s)_n|, Gershgorin radius, max |b|,
                             // max |b - A x0| of the level solve, max |b| over levels 0..n (bit patterns)
  double tgt;              // residual reduction asked of a level solve
  double ntol;             // a third of the Newton tolerance (the last step's linear residual)
  int kcap;                // at most this many iterations (the launches the host issues)
};

// Chebyshev for a spectrum in [a, b]: d_0 = z_0 / theta; d_k = rho_k rho_{k-1} d_{k-1} +
// (2 rho_k / delta) z_k, rho_0 = delta / theta, rho_k = 1 / (2 theta / delta - rho_{k-1}).
// Returns the iterations that reach `target` (error bound 2 q^K, q = (sqrt(b/a) - 1) / (sqrt(b/a) + 1)).
__host__ __device__ inline int cheb_coefficients(double a, double b, double target, float2* c) {
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
  const double q = (sqrt(b / a) - 1.0) / (sqrt(b / a) + 1.0);
  int K = q > 0 ? (int)ceil(log(0.5 * target) / log(q)) : 1;
  K = K < 1 ? 1 : (K > kMaxCheb ? kMaxCheb : K);
  double rho = delta / theta;
  c[0] = make_float2(0.f, (float)(1.0 / theta));
  for (int k = 1; k < K; ++k) {
    const double rn = 1.0 / (2.0 * theta / delta - rho);
    c[k] = make_float2((float)(rn * rho), (float)(2.0 * rn / delta));
    rho = rn;
  }
  return K;
}

// Chebyshev plan of a multigrid-preconditioned level solve whose iterate has max |u| = umax:
// with M = I + tau mu_a (-Delta_h) the spectrum of M^{-1} A lies near [1, mu(umax) / mu_a];
// the V-cycle B moves the lower end to kMgLow. The upper end is taken at mu(1.05 umax) and
// widened by 5 % for the non-symmetric mu' terms of the Jacobian and float32 rounding.
// (Measured for the heat Jacobian at max |u| = 1, N = 66, 127, 255: spec(B A) is real and lies
// in [0.82, 2.0], against the planned [0.75, 2.21].)
__host__ __device__ inline int mg_cheb_plan(double mu_a, double mu_b, double umax, double target, float2* c) {
  const double um = 1.05 * umax;
  const double ratio = (mu_a + mu_b * um * um) / mu_a;
  return cheb_coefficients(kMgLow, 1.05 * ratio, target, c);
}

// out[n] = max |U^n| (bit pattern of a non-negative double), one work-group per level
__global__ __launch_bounds__(256) void k_level_absmax(const double* __restrict__ U, size_t ns,
                                                      unsigned long long* __restrict__ out) {
  const double* u = U + (size_t)blockIdx.x * ns;
  double m = 0.0;
  for (size_t i = threadIdx.x; i < ns; i += 256) m = nanmax(m, fabs(u[i]));
  m = wave_max(m);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = __double_as_longlong(nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3])));
}

// Work items (lane, tile of 64 x 32 nodes), sorted by level count; thread (c, g) of the
// 64 x 4 work-group walks kPcRows rows of column c, keeping the column's u and x of the rows
// above and below in registers. Iteration k of level n: r = b - A x with b = r^n + du^{n-1}
// (Eq. (7)) and x = du^n (x = 0 at k = 0, written here; b replaces r^n then, so that later
// iterations read one array for it). m: the level (bulk) or the diagonal (pipelined); the
// lane's level is m - stage.
constexpr int kPcRows = 8, kPcTileY = 4 * kPcRows;
__host__ __device__ inline int pc_tiles(int nx, int ny) { return ((nx + 63) / 64) * ((ny + kPcTileY - 1) / kPcTileY); }
// Column (x, rows y0..y1-1) of k_pc_resid; XT: the type of the iterate x and of du^{n-1}.
// With warm (the pipelined lanes, n > 0) the first iteration starts from x0 = du^{n-1}: it
// writes x = x0 and r = b - A x0, and returns max |b| and max |r| of the column in bm, rm.
template <typename XT>
__device__ __forceinline__ void pc_resid_column(const PcDesc* d, const KProb& p, int n, int k, int x, int y0, int y1,
                                                XT* __restrict__ X, const XT* __restrict__ prev, bool warm,
                                                double& bm, double& rm) {
  const int nx = p.nx, ny = p.ny;
  const unsigned ns = (unsigned)nx * (unsigned)ny;
  double* __restrict__ R = d->R + (size_t)(n & d->rmask) * ns;
  float* __restrict__ r = d->r;
  if (k == 0 && !warm) {  // b = r^n + du^{n-1} is kept in place of r^n for the later iterations
    for (int y = y0; y < y1; ++y) {
      const unsigned i = (unsigned)y * nx + x;
      const double b = R[i] + (prev ? (double)prev[i] : 0.0);
      R[i] = b;
      X[i] = (XT)0;
      r[(size_t)y * d->ld + x] = (float)b;
      bm = nanmax(bm, fabs(b));
      rm = nanmax(rm, fabs(b));
    }
    return;
  }
  // the iterate the residual is formed from: x, or x0 = du^{n-1} at a warm first iteration
  // (read from du^{n-1}, which no thread writes here; x is set to it alongside)
  const XT* __restrict__ Xr = (k == 0) ? prev : X;
  const double* __restrict__ Un = d->U + (size_t)n * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
  double uS = node_value(p, Un, bd, x, y0 - 1), uP = Un[(unsigned)y0 * nx + x];
  double xS = y0 > 0 ? (double)Xr[(unsigned)(y0 - 1) * nx + x] : 0.0, xP = (double)Xr[(unsigned)y0 * nx + x];
  for (int y = y0; y < y1; ++y) {
    const unsigned i = (unsigned)y * nx + x;
    const double uN = y + 1 < ny ? Un[i + nx] : node_value(p, Un, bd, x, y + 1);
    const double xN = y + 1 < ny ? (double)Xr[i + nx] : 0.0;
    Nb u;
    u.P = uP;
    u.S = uS;
    u.N = uN;
    u.W = x > 0 ? Un[i - 1] : node_value(p, Un, bd, x - 1, y);
    u.E = x + 1 < nx ? Un[i + 1] : node_value(p, Un, bd, x + 1, y);
    Row5 a;
    (void)eval_point<0, kFormNoConv>(p, u, x, y, a);  // these solves are for heat only (no convection)
    double ax = a.C * xP;
    if (x > 0) ax += a.W * (double)Xr[i - 1];
    if (x < nx - 1) ax += a.E * (double)Xr[i + 1];
    if (y > 0) ax += a.S * xS;
    if (y < ny - 1) ax += a.N * xN;
    double b = R[i];
    if (k == 0) {  // warm first iteration
      b += xP;
      R[i] = b;
      X[i] = Xr[i];
      bm = nanmax(bm, fabs(b));
      rm = nanmax(rm, fabs(b - ax));
    }
    r[(size_t)y * d->ld + x] = (float)(b - ax);
    uS = uP;
    uP = uN;
    xS = xP;
    xP = xN;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_pc_resid(const PcDesc* __restrict__ ds, const int2* __restrict__ items,
                                                   int m, int k, int count) {
  const unsigned wi = xcd_band(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
  if (wi >= (unsigned)count) return;
  const int2 it = items[wi];
  const PcDesc* d = ds + it.x;
  const int n = m - d->stage;
  // iteration 0 runs before the lanes plan their iteration counts (pipelined) or with them
  if (!d->active || n < 0 || n >= d->p.nt || (k > 0 && k >= d->K[n])) return;
  const KProb p = at_level(d->p, n);
  const int nx = p.nx, ny = p.ny, tilesx = (nx + 63) >> 6;
  const int x = (it.y % tilesx) * 64 + (threadIdx.x & 63);
  const int y0 = (it.y / tilesx) * kPcTileY + (threadIdx.x >> 6) * kPcRows, y1 = min(y0 + kPcRows, ny);
  const unsigned ns = (unsigned)nx * (unsigned)ny;
  double bm = 0.0, rm = 0.0;
  if (x < nx && y0 < ny) {
    if (d->dxf)
      pc_resid_column<float>(d, p, n, k, x, y0, y1, d->dxf + (size_t)(n & 1) * ns,
                             n > 0 ? d->dxf + (size_t)((n - 1) & 1) * ns : nullptr, n > 0, bm, rm);
    else
      pc_resid_column<double>(d, p, n, k, x, y0, y1, d->dU + (size_t)(n & d->dmask) * ns,
                              n > 0 ? d->dU + (size_t)((n - 1) & d->dmask) * ns : nullptr, false, bm, rm);
  }
  if (k != 0 || !d->dxf) return;  // uniform over the work-group
  // the first iteration of a pipelined lane: max |b| and max |b - A x0| of the level
  __shared__ double red[2][4];
  bm = wave_max(bm);
  rm = wave_max(rm);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = bm;
    red[1][threadIdx.x >> 6] = rm;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const double* q = red[threadIdx.x];
    atomic_max_nonneg(d->stat + kStat * (size_t)n + 3 + threadIdx.x, nanmax(nanmax(q[0], q[1]), nanmax(q[2], q[3])));
  }
}

// V-cycle launches of iteration k of level n. Items (lane, grid l, tile x, tile y) of the
// lanes that have level n; lanes without level n or iteration k return.
__global__ __launch_bounds__(kMgThreads) void k_mg_down(const MgDesc* __restrict__ mg, const PcDesc* __restrict__ ds,
                                                 const int4* __restrict__ items, int m, int k, int count) {
  const unsigned wi = xcd_band(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
  if (wi >= (unsigned)count) return;
  const int4 it = items[wi];
  const PcDesc* d = ds + it.x;
  const int n = m - d->stage;
  if (!d->active || n < 0 || n >= d->p.nt || k >= d->K[n]) return;
  // the x-restriction (T, kMgDS x kMgTC) reuses X, which is dead once the residual is formed
  static_assert(kMgTC <= kMgDS, "T fits in X");
  __shared__ float F[kMgDS * kMgDS], X[kMgDS * kMgDS];
  __shared__ MgDownAux aux;
  mg_down_tile(mg[it.x], it.y, it.z, it.w, F, X, X, aux);
}

// The Chebyshev step of iteration k at node (i, j), given z = B r there: d = c0 d + c1 z in
// float32, du^n += d (FP64 in the bulk schedule, float32 in a pipelined lane's ring). Applied
// by the V-cycle's last kernel on the finest grid.
struct ChebStep {
  const PcDesc* d;
  int n, k, N;
  __device__ void operator()(int i, int j, float z) const {
    const size_t idx = (size_t)j * N + i;
    const float2 c = d->c[(size_t)n * kMaxCheb + k];
    const float dir = (k == 0 ? 0.f : c.x * d->d[idx]) + c.y * z;
    d->d[idx] = dir;
    if (d->dxf)
      d->dxf[(size_t)(n & 1) * N * N + idx] += dir;
    else
      d->dU[(size_t)(n & d->dmask) * N * N + idx] += (double)dir;
  }
};

__global__ __launch_bounds__(kMgThreads) void k_mg_up(const MgDesc* __restrict__ mg, const PcDesc* __restrict__ ds,
                                               const int4* __restrict__ items, int m, int k, int count) {
  const unsigned wi = xcd_band(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
  if (wi >= (unsigned)count) return;
  const int4 it = items[wi];
  const PcDesc* d = ds + it.x;
  const int n = m - d->stage;
  if (!d->active || n < 0 || n >= d->p.nt || k >= d->K[n]) return;
  __shared__ float X[kMgUS * kMgUS], X1[kMgUS * kMgUS], E[kMgUE * kMgUE];
  const MgDesc& mg_ = mg[it.x];
  const int l = it.y;
  if (l == 0) {
    mg_up_tile(mg_, 0, it.z, it.w, X, X1, E, ChebStep{d, n, k, mg_.n[0]});
  } else {
    float* e = mg_.e[l];
    const int nl = mg_.n[l];
    mg_up_tile(mg_, l, it.z, it.w, X, X1, E, [=](int i, int j, float v) { e[(size_t)j * nl + i] = v; });
  }
}

// One work-group per lane: the V-cycle's grids from G down (LDS).
__global__ __launch_bounds__(1024) void k_mg_lds(const MgDesc* __restrict__ mg, const PcDesc* __restrict__ ds,
                                                 const int* __restrict__ items, int m, int k) {
  const int i = items[blockIdx.x];
  const PcDesc* d = ds + i;
  const int n = m - d->stage;
  if (!d->active || n < 0 || n >= d->p.nt || k >= d->K[n]) return;
  __shared__ float X[kMgLdsWords], F[kMgLdsWords], T[kMgLdsWords];
  const MgDesc& mg_ = mg[i];
  if (mg_.G == 0) {
    mg_lds_cycle(mg_, X, F, T, ChebStep{d, n, k, mg_.n[0]});
  } else {
    float* x = mg_.x[mg_.G];
    const int nl = mg_.n[mg_.G];
    mg_lds_cycle(mg_, X, F, T, [=](int a, int b, float v) { x[b * nl + a] = v; });
  }
}

// ---------------------------------------------- pipelined Newton stages (multigrid lanes)
// Newton stage s at level n needs U^(s) at levels n and n-1 and du^(s) of level n-1; it
// produces du^(s)_n, from which U^(s+1)_n = U^(s)_n + du^(s)_n. Stage s therefore runs on
// level n at diagonal D = n + s: lane s of an instance applies the update of stage s-1 to level
// n (k_pipe_update), forms r^(s)_n (k_pipe_residual), plans its Chebyshev iteration from
// max |U^(s)_n| (k_pipe_cheb) and solves (k_pc_resid and the V-cycle launches), all in the
// launches of diagonal D. Lane s-1 works on level n+1 at the same diagonal and needs the
// U^(s-1)_n that lane s overwrites: lane s parks it first. Lane S (after the last stage) only
// updates and forms the residual of the result. The update rings hold two levels: du^(s)_n is
// read at diagonal D+1 (by lane s at level n+1 and by lane s+1 at level n) and overwritten at
// D+2.
__global__ __launch_bounds__(256) void k_pipe_update(const PcDesc* __restrict__ ds, const int2* __restrict__ items,
                                                      int D, int count) {
  const unsigned wi = xcd_band(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
  if (wi >= (unsigned)count) return;
  const int2 it = items[wi];
  const PcDesc* d = ds + it.x;
  const int n = D - d->stage;
  if (!d->active || d->stage == 0 || n < 0 || n >= d->p.nt) return;
  const int nx = d->p.nx, ny = d->p.ny, tilesx = (nx + 63) >> 6;
  const int x = (it.y % tilesx) * 64 + (threadIdx.x & 63);
  const int y0 = (it.y / tilesx) * kPcTileY + (threadIdx.x >> 6) * kPcRows, y1 = min(y0 + kPcRows, ny);
  if (x >= nx) return;
  const unsigned ns = (unsigned)nx * (unsigned)ny;
  double* __restrict__ u = d->U + (size_t)n * ns;
  const float* __restrict__ du = d->dprev + (size_t)(n & 1) * ns;
  for (int y = y0; y < y1; ++y) {
    const unsigned i = (unsigned)y * nx + x;
    const double old = u[i];
    d->park_out[i] = old;
    u[i] = old + (double)du[i];
  }
}

// r^(s)_n = -(U^(s)_n - U^(s)_{n-1} + tau F(U^(s)_n)) into the lane's level buffer, with
// max |U^(s)_n|, max |r| and the Gershgorin radius of the level's rows into stat[n]
// (tiles as k_pc_resid, the column's u of the rows above and below kept in registers).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_pipe_residual(const PcDesc* __restrict__ ds, const int2* __restrict__ items,
                                                        int D, int count) {
  const unsigned wi = xcd_band(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
  if (wi >= (unsigned)count) return;
  const int2 it = items[wi];
  const PcDesc* d = ds + it.x;
  const int n = D - d->stage;
  if (!d->active || n < 0 || n >= d->p.nt) return;
  const KProb p = at_level(d->p, n);
  const int nx = p.nx, ny = p.ny, tilesx = (nx + 63) >> 6;
  const int x = (it.y % tilesx) * 64 + (threadIdx.x & 63);
  const int y0 = (it.y / tilesx) * kPcTileY + (threadIdx.x >> 6) * kPcRows, y1 = min(y0 + kPcRows, ny);
  const unsigned ns = (unsigned)nx * (unsigned)ny;
  double uabs = 0.0, rabs = 0.0, rho = 0.0;
  if (x < nx && y0 < ny) {
    const double* __restrict__ Un = d->U + (size_t)n * ns;
    const double* __restrict__ up = n == 0 ? d->u0 : (d->park_in ? d->park_in : d->U + (size_t)(n - 1) * ns);
    const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
    double uS = node_value(p, Un, bd, x, y0 - 1), uP = Un[(unsigned)y0 * nx + x];
    for (int y = y0; y < y1; ++y) {
      const unsigned i = (unsigned)y * nx + x;
      Nb u;
      u.P = uP;
      u.S = uS;
      u.N = y + 1 < ny ? Un[i + nx] : node_value(p, Un, bd, x, y + 1);
      u.W = x > 0 ? Un[i - 1] : node_value(p, Un, bd, x - 1, y);
      u.E = x + 1 < nx ? Un[i + 1] : node_value(p, Un, bd, x + 1, y);
      Row5 a;
      const double F = eval_point<0, kFormNoConv>(p, u, x, y, a);
      const double r = -(u.P - up[i] + p.dt * F);
      if (!d->last) d->R[i] = r;
      uabs = nanmax(uabs, fabs(u.P));
      rabs = nanmax(rabs, fabs(r));
      rho = nanmax(rho, gersh(a));
      uS = uP;
      uP = u.N;
    }
  }
  __shared__ double red[3][4];
  uabs = wave_max(uabs);
  rabs = wave_max(rabs);
  rho = wave_max(rho);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = uabs;
    red[1][w] = rabs;
    red[2][w] = rho;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const double* q = red[threadIdx.x];
    atomic_max_nonneg(d->stat + kStat * (size_t)n + threadIdx.x, nanmax(nanmax(q[0], q[1]), nanmax(q[2], q[3])));
  }
}

// Chebyshev plan of each solving lane's level (one thread per lane); kq[q]: the iterations
// lane q runs at this diagonal (0 without a level).
__global__ __launch_bounds__(64) void k_pipe_cheb(const PcDesc* __restrict__ ds, const int* __restrict__ lanes, int nl,
                                                  int D, int* __restrict__ kq) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= nl) return;
  const PcDesc* d = ds + lanes[q];
  const int n = D - d->stage;
  if (!d->active || d->last || n < 0 || n >= d->p.nt) {
    kq[q] = 0;
    return;
  }
  unsigned long long* st = d->stat + kStat * (size_t)n;
  const double umax = __longlong_as_double((long long)st[0]);
  // the solve starts from x0 = du^{n-1} (k_pc_resid): it has to reduce |b - A x0| to tgt |b|
  const double bmax = __longlong_as_double((long long)st[3]), r0 = __longlong_as_double((long long)st[4]);
  // max |b| over this lane's levels so far (level n-1's entry: written by this thread's lane at
  // the previous diagonal)
  const double run = n > 0 ? fmax(bmax, __longlong_as_double((long long)st[5 - kStat])) : bmax;
  st[5] = (unsigned long long)__double_as_longlong(run);
  double tgt = d->tgt;
  // where the reduction asked leaves a linear residual tgt max|b| within a factor 10 of tol over
  // all of the lane's levels so far, this Newton step can be the instance's last: each level
  // solves to ntol instead (at most 10x tighter), so that the step's result meets tol rather than
  // missing it narrowly and taking one more step
  if (bmax > 0.0 && d->ntol > 0.0 && 10.0 * d->ntol >= d->tgt * run) tgt = fmin(tgt, d->ntol / bmax);
  if (r0 > 0.0 && bmax > 0.0) tgt = fmin(0.5, tgt * bmax / r0);
  int K = mg_cheb_plan(d->p.mu_a, d->p.mu_b, umax, tgt, d->c + (size_t)n * kMaxCheb);
  K = K < d->kcap ? K : d->kcap;
  d->K[n] = K;
  kq[q] = K;
}

// ---------------------------------------------------------- wavefront schedule
// Newton iteration j at level n needs the iterate U_j at level n (written by iteration
// j-1) and U_{j+1}^{n-1} = U_j^{n-1} + du_j^{n-1} (iteration j, level n-1). All pairs (j, n)
// on the anti-diagonal n + 2j = diag are therefore independent and run in one launch; the
// launch order d = 0, 1, 2, ... carries every dependency, and no two pairs of one launch
// touch the same level of the same buffer. Pair (j, n) forms the rows of A_n(U_j) and the
// right-hand side of Eq. (7), r_j^n + du_j^{n-1} = -(U_j^n - U_{j+1}^{n-1} + tau F(U_j^n))
// (the -I block moves du_j^{n-1} into the time difference, so the update itself is never
// stored), solves A_n du_j^n = that on its tile, writes U_{j+1}^n = U_j^n + du_j^n, and from
// the tile's U_{j+1} also the next iterate's residual r_{j+1}^n and Gershgorin radius. The
// radius of level n fixes the Chebyshev interval of stage j+1 at that level: each tile
// leaves its value in a slot of its own (a ring of four levels per stage, read two
// anti-diagonals later and overwritten four later), and the consuming pair takes the
// maximum. The residual maxima go to one running slot per (stage, tile), folded after the
// sequence (k_stage_max). Plain stores throughout: every slot has one writer at a time.
// Per node and pair: U_j^n and U_{j+1}^{n-1} read, U_{j+1}^n written.
struct WaveArgs {
  double* Ur[2];                  // iterate ring: stage j reads Ur[j & 1], writes Ur[(j + 1) & 1]
  const double* u0;               // initial condition (level 0)
  const double* rho_in;           // radius of A_n(U_0) at rho_in[2n + 1] (bit pattern)
  double* rho_part;               // [stages + 1][4][tiles]: radius of A_n(U_j) on a tile, slot n % 4
  double* res_part;               // [stages + 1][tiles]: running max |r(U_j)| of a tile (zero at start)
  int tiles;                      // tiles per level
  int stages;
};

// The pair (stage j, level n = diag - 2j) on one tile; nothing when n is outside the levels.
template <typename T, int BC, int FORM>
__device__ __forceinline__ void wave_pair(const KProb& p, const WaveArgs& a, const Geo& g, int j, int tile, int diag,
                                          int passes, int sweeps) {
  __shared__ double lds_raw[2 * kWaves * 2 * 64];
  __shared__ double om[kMaxSweeps];
  __shared__ double red[2][kWaves];
  // U_j^n and U_{j+1}^{n-1} of the region parked in LDS while the inner solve runs (they
  // are needed again only afterwards; kept in registers they would spill)
  __shared__ double park[2][kRows][kThreads];
  const int n = diag - 2 * j;
  if (n < 0 || n >= p.nt) return;  // uniform over the work-group
  const int lane = threadIdx.x & 63;
  // wave index as a wave-uniform value: row indices, their products with the row stride and
  // the periodic wrap of rows are then scalar work
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = tile % g.tilesx, ty = tile / g.tilesx;
  const int rx0 = g.whole ? 0 : tx * g.TX - g.H;
  const int ry0 = g.whole ? 0 : ty * g.TY - g.H;
  const size_t ns = (size_t)p.nx * p.ny;
  const double* un = a.Ur[j & 1] + (size_t)n * ns;
  // U_{j+1}^{n-1}, stored by the pair (j, n-1) on the previous anti-diagonal (u^0 at n = 0)
  const double* upn_in = n == 0 ? a.u0 : a.Ur[(j + 1) & 1] + (size_t)(n - 1) * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
  if (wave == 0) {  // radius of A_n(U_j): the residual kernel's at j = 0, else the tiles' maximum
    double rho_j = 0.0;
    if (j == 0) {
      rho_j = a.rho_in[2 * n + 1];
    } else {
      const double* rp = a.rho_part + ((size_t)j * 4 + (n & 3)) * a.tiles;
      for (int t = lane; t < a.tiles; t += 64) rho_j = max_nn(rho_j, rp[t]);
      rho_j = wave_max_nn(rho_j);
    }
    cheb_table(om, clamp_rho(rho_j), sweeps);
  }

  RegionSolve<T> rs;
  double uc[kRows], upn[kRows];  // U_j^n and U_{j+1}^{n-1} at the region nodes
  unsigned idx[kRows];
  const int gx = rx0 + lane;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    int x, y;
    const bool act = region_node<BC>(p, gx, ry0 + wave * kRows + k, x, y);
    idx[k] = act ? (unsigned)y * (unsigned)p.nx + x : ~0u;
    Row5 r5;
    if (act) {
      const Nb u = gather<BC>(p, un, bd, x, y);
      const double F = eval_point<BC, FORM>(p, u, x, y, r5);
      const double prev = ld(upn_in, idx[k]);
      rs.bb[k] = -(u.P - prev + p.dt * F);
      uc[k] = u.P;
      upn[k] = prev;
      // (periodic only: Dirichlet boundary rows drop neighbours the folded form would keep)
      if constexpr (BC == 1 && FORM == kFormConstVisc)
        rs.set_row_const_visc(k, p, u, r5);
      else
        rs.set_row(k, r5, FORM == kFormConstVisc ? p.ic0 : 1.0 / r5.C);
    } else {
      r5.C = 1.0;
      r5.W = r5.E = r5.S = r5.N = 0.0;
      rs.bb[k] = 0.0;
      uc[k] = 0.0;
      upn[k] = 0.0;
      rs.set_row(k, r5, 1.0);
    }
    rs.X[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    park[0][k][threadIdx.x] = uc[k];
    park[1][k][threadIdx.x] = upn[k];
  }
  __syncthreads();  // omega table
  rs.run(passes, sweeps, false, om, lds_raw, wave, lane);

  // U_{j+1} on the region (valid one node beyond the tile), its neighbours, and the
  // residual and radius of the next iterate on the tile
  double unew[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    unew[k] = park[0][k][threadIdx.x] + rs.X[k];
    upn[k] = park[1][k][threadIdx.x];
  }
  int par = 0;
  const YNb<double> yn = y_exchange<double>(unew, lds_raw, par, wave, lane);
  double rmax = 0.0, gmax = 0.0;
  double* Uo = a.Ur[(j + 1) & 1] + (size_t)n * ns;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    Nb u;
    u.P = unew[k];
    u.S = k == 0 ? yn.s0 : unew[k - 1];
    u.N = k == kRows - 1 ? yn.nM : unew[k + 1];
    u.W = lane_from_left(unew[k]);
    u.E = lane_from_right(unew[k]);
    const int row = wave * kRows + k;
    const int gy = ry0 + row;
    if (idx[k] != ~0u && in_tile(g, p, lane, row, gx, gy)) {
      const int x = gx, y = gy;
      if (BC == 0) {  // Dirichlet neighbours outside the domain are data
        if (x == 0) u.W = node_value(p, un, bd, -1, y);
        if (x == p.nx - 1) u.E = node_value(p, un, bd, p.nx, y);
        if (y == 0) u.S = node_value(p, un, bd, x, -1);
        if (y == p.ny - 1) u.N = node_value(p, un, bd, x, p.ny);
      }
      Row5 q;
      const double F = eval_point<BC, FORM>(p, u, x, y, q);
      const double r = -(u.P - upn[k] + p.dt * F);
      // |r| and the radius are >= 0 or NaN with a clear sign bit (max_nn applies)
      rmax = max_nn(rmax, fabs(r));
      gmax = max_nn(gmax, FORM == kFormConstVisc ? gersh(q, p.ic0) : gersh(q));
      st(Uo, idx[k], unew[k]);
    }
  }
  rmax = wave_max_nn(rmax);
  gmax = wave_max_nn(gmax);
  if (lane == 0) {
    red[0][wave] = rmax;
    red[1][wave] = gmax;
  }
  __syncthreads();
  static_assert(kWaves == 16, "the fold of the wave maxima is one row of 16 lanes");
  if (wave == 0) {  // the kWaves wave maxima, folded across the first row's lanes
    const double r = lane_value(row_max_nn(lane < kWaves ? red[0][lane] : 0.0), 0);
    const double q = lane_value(row_max_nn(lane < kWaves ? red[1][lane] : 0.0), 0);
    if (lane == 0) {
      double* rs = a.res_part + (size_t)(j + 1) * a.tiles + tile;
      *rs = max_nn(*rs, r);
      a.rho_part[((size_t)(j + 1) * 4 + (n & 3)) * a.tiles + tile] = q;
    }
  }
}

// One launch per anti-diagonal: grid = stages x tiles per level, blockIdx.x = j * tiles + tile.
template <typename T, int BC, int FORM>
__global__ __launch_bounds__(kThreads) void k_level_wave(KProb p, WaveArgs a, Geo g, int diag, int passes,
                                                         int sweeps) {
  const int tiles_per_level = gridDim.x / a.stages;
  wave_pair<T, BC, FORM>(p, a, g, blockIdx.x / tiles_per_level, blockIdx.x % tiles_per_level, diag, passes,
                         sweeps);
}

// The whole sequence in one cooperative launch (every work-group resident): work-group
// (j, tile) takes its pair on each anti-diagonal in turn, and a grid barrier separates
// consecutive anti-diagonals, in place of the kernel boundary. bar[0] counts arrivals (zero
// at launch), bar[1] is set when a barrier wait exceeds spin_limit polls: every work-group
// then leaves, the sequence is incomplete and the host reports it. Before arriving, each wave
// waits for its stores and one release fence per work-group writes the XCD's L2 back, making
// them visible to the other XCDs; after the wait one acquire fence per work-group drops stale
// lines before the next anti-diagonal reads its neighbours' data. (Fences in every thread
// would repeat the L2 write-back and invalidation once per wave.)
template <typename T, int BC, int FORM>
__global__ __launch_bounds__(kThreads) void k_level_wave_seq(KProb p, WaveArgs a, Geo g, int ndiag, int passes,
                                                             int sweeps, unsigned* bar, unsigned spin_limit) {
  __shared__ int stop;
  const int tiles_per_level = gridDim.x / a.stages;
  const int j = blockIdx.x / tiles_per_level, tile = blockIdx.x % tiles_per_level;
  for (int d = 0; d < ndiag; ++d) {
    // j and tile pass through an empty asm statement, so the pair's region indices are formed
    // anew on every anti-diagonal rather than hoisted out of the loop and held in registers
    int jj = j, tt = tile;
    asm volatile("" : "+s"(jj), "+s"(tt));
    wave_pair<T, BC, FORM>(p, a, g, jj, tt, d, passes, sweeps);
    if (d + 1 == ndiag) break;
    // every wave waits until its stores have reached the L2 (all counters to zero); then one
    // thread writes the XCD's L2 back (it holds the stores of all waves) and arrives
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __builtin_amdgcn_s_waitcnt(0);  // the write-back has completed before the arrival
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = (unsigned)(d + 1) * gridDim.x;
      int quit = 0;
      for (unsigned spins = 0;
           __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++spins) {
        if (spins >= spin_limit || __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          quit = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (quit) __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // invalidates the XCD's L2 and this compute unit's L1, which all waves read through,
      // complete before the other waves pass the work-group barrier
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
      stop = quit;
    }
    __syncthreads();
    if (stop) return;
  }
}

// ------------------------------------------------------------ batched wavefront
// Instances of one problem (same sizes, coefficients and boundary data; own initial
// conditions and iterates) share each anti-diagonal launch: grid (stages x tiles,
// instances), blockIdx.y selects the instance's arguments. Every instance runs the same
// stage count, so a launch carries all of their pairs of that anti-diagonal.
template <typename T, int BC, int FORM>
__global__ __launch_bounds__(kThreads) void k_level_wave_batch(KProb p, const WaveArgs* __restrict__ as, Geo g,
                                                               int diag, int passes, int sweeps) {
  const WaveArgs a = as[blockIdx.y];
  const int tiles_per_level = gridDim.x / a.stages;
  wave_pair<T, BC, FORM>(p, a, g, blockIdx.x / tiles_per_level, blockIdx.x % tiles_per_level, diag, passes,
                         sweeps);
}

// ------------------------------------------------------------ Theorem 1 windows
// y = A_m x at every node of level m (rows from U_m, Eq. (6)); products P^{w-1} r^w of
// the Section 5 recursion are chains of these. One thread per node.
template <int BC>
__global__ __launch_bounds__(256) void k_apply(KProb p0, int m, const double* __restrict__ U,
                                               const double* __restrict__ x, double* __restrict__ y) {
  const KProb p = at_level(p0, m);
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  const unsigned ns = (unsigned)p.nx * (unsigned)p.ny;
  if (i >= ns) return;
  const int xi = (int)(i % (unsigned)p.nx), yi = (int)(i / (unsigned)p.nx);
  const double* um = U + (size_t)m * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)m * 2 * (p.nx + p.ny) : nullptr;
  const Nb u = gather<BC>(p, um, bd, xi, yi);
  Row5 a;
  (void)eval_point<BC>(p, u, xi, yi, a);
  // neighbour values of x (periodic wrap; absent Dirichlet columns have zero rows)
  const Nb v = gather<BC>(p, x, nullptr, xi, yi);
  y[i] = a.C * v.P + a.W * v.W + a.E * v.E + a.S * v.S + a.N * v.N;
}

// z = x + y (n values); y may be NULL (copy).
__global__ __launch_bounds__(256) void k_add(size_t n, const double* __restrict__ x, const double* __restrict__ y,
                                             double* __restrict__ z) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    z[i] = x[i] + (y ? y[i] : 0.0);
}

// ------------------------------------------------------------------- update
__global__ __launch_bounds__(256) void k_update(size_t count, double* __restrict__ U,
                                                const double* __restrict__ dU, double* __restrict__ partial) {
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const double d = dU[i];
    U[i] += d;
    acc += d * d;
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Fixed-order sum of `count` partials into out[0] (one block).
__global__ __launch_bounds__(256) void k_reduce_sum(const double* __restrict__ partial, int count,
                                                    double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = max |a[i]| over count values (one block, fixed order; NaN propagates).
__global__ __launch_bounds__(256) void k_absmax(const double* __restrict__ a, size_t count,
                                                unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (size_t i = threadIdx.x; i < count; i += blockDim.x) {
    const double v = a[i];
    m = nanmax(m, fabs(v));
  }
  m = wave_max(m);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
    out[0] = __double_as_longlong(r);
  }
}

// out[k] = max_t part[k][t] over `tiles` slots for k = 0..stages (one block per k; NaN
// propagates): the residual maxima of a wavefront sequence.
__global__ __launch_bounds__(256) void k_stage_max(const double* __restrict__ part, int tiles,
                                                   double* __restrict__ out) {
  const double* pk = part + (size_t)blockIdx.x * tiles;
  double m = 0.0;
  for (int t = threadIdx.x; t < tiles; t += 256) m = nanmax(m, pk[t]);
  m = wave_max(m);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

// part[b] = max over the block's points p of max_n |sum_{m<=n} R[m][p]| (NaN propagates):
// the block forward substitution of Eq. (7) with identity diagonal blocks. 64-thread work-
// groups, grid-stride over the ns points of a level, levels read four at a time; fold part
// with k_absmax.
__global__ __launch_bounds__(64) void k_cumsum_absmax(size_t ns, int nt, const double* __restrict__ R,
                                                      double* __restrict__ part) {
  double m = 0.0;
  for (size_t i = (size_t)blockIdx.x * 64 + threadIdx.x; i < ns; i += (size_t)gridDim.x * 64) {
    double acc = 0.0;
    int n = 0;
    for (; n + 4 <= nt; n += 4) {
      const double r0 = R[(size_t)n * ns + i], r1 = R[(size_t)(n + 1) * ns + i];
      const double r2 = R[(size_t)(n + 2) * ns + i], r3 = R[(size_t)(n + 3) * ns + i];
      acc += r0;
      m = nanmax(m, fabs(acc));
      acc += r1;
      m = nanmax(m, fabs(acc));
      acc += r2;
      m = nanmax(m, fabs(acc));
      acc += r3;
      m = nanmax(m, fabs(acc));
    }
    for (; n < nt; ++n) {
      acc += R[(size_t)n * ns + i];
      m = nanmax(m, fabs(acc));
    }
  }
  m = wave_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Accumulated-residual norm max_{n,p} |sum_{m<=n} r^m_p| of an iterate without storing R, in
// two passes. Pass 1 (grid: points x chunks of kJudgeLevels levels): per point, the residuals
// r^n = -(u^n - u^{n-1} + tau F(u^n)) of the chunk's levels, their total and the largest and
// smallest partial sum inside the chunk -> tot, hi, lo [chunk][point]. Pass 2: per point, the
// prefix P of the earlier chunks gives max |P + s| over the chunk's partial sums s as
// max(|P + hi|, |P + lo|); block maxima -> part (fold with k_absmax). NaN propagates.
constexpr int kJudgeLevels = 16;
template <int BC>
__global__ __launch_bounds__(256) void k_judge_chunks(KProb p, const double* __restrict__ U,
                                                      const double* __restrict__ u0, double* __restrict__ tot,
                                                      double* __restrict__ hi, double* __restrict__ lo) {
  const unsigned ns = (unsigned)p.nx * (unsigned)p.ny;
  // gridDim.x is the fast index of the linear id, so a multiple of 8 keeps bands per XCD
  const unsigned i = xcd_band(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (i >= ns) return;
  const int x = (int)(i % (unsigned)p.nx), y = (int)(i / (unsigned)p.nx);
  const int c = blockIdx.y, n0 = c * kJudgeLevels, n1 = min(p.nt, n0 + kJudgeLevels);
  double acc = 0.0, mx = -__longlong_as_double(0x7ff0000000000000ll), mn = -mx;
  // levels four at a time: all neighbour loads of a group are issued before its arithmetic
  for (int g = n0; g < n1; g += 4) {
    Nb u[4];
    double prev[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int n = min(g + k, n1 - 1);
      const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (p.nx + p.ny) : nullptr;
      u[k] = gather<BC>(p, U + (size_t)n * ns, bd, x, y);
      prev[k] = (n == 0 ? u0 : U + (size_t)(n - 1) * ns)[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (g + k < n1) {
        Row5 r5;
        const double F = eval_point<BC>(p, u[k], x, y, r5);
        acc += -(u[k].P - prev[k] + p.dt * F);
        mx = acc > mx || acc != acc ? acc : mx;
        mn = acc < mn || acc != acc ? acc : mn;
      }
    }
  }
  const size_t o = (size_t)c * ns + i;
  tot[o] = acc;
  hi[o] = mx;
  lo[o] = mn;
}

__global__ __launch_bounds__(256) void k_judge_fold(size_t ns, int nchunks, const double* __restrict__ tot,
                                                    const double* __restrict__ hi, const double* __restrict__ lo,
                                                    double* __restrict__ part) {
  double m = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (size_t)gridDim.x * blockDim.x) {
    double P = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      const size_t o = (size_t)c * ns + i;
      m = nanmax(m, nanmax(fabs(P + hi[o]), fabs(P + lo[o])));
      P += tot[o];
    }
  }
  m = wave_max(m);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

// Judge of the learned initial iterate, decided on the device: with rp = max|R| of the
// prediction already in U (bits at scal[0]) and r0 = mult * max|R| of the plain iterate
// (bits at scal[2]), U keeps the prediction if rp is finite and rp < r0, else U <- u^0 at
// every level. Every thread evaluates the same decision.
__global__ __launch_bounds__(256) void k_judge_apply(size_t ns, int nt, double* __restrict__ U,
                                                     const double* __restrict__ u0,
                                                     const unsigned long long* __restrict__ scal, double mult) {
  const double rp = __longlong_as_double(scal[0]);
  const double r0 = __longlong_as_double(scal[2]) * mult;
  if (isfinite(rp) && rp < r0) return;
  const size_t total = ns * (size_t)nt;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
    U[i] = u0[i % ns];
}

// u^n = u^0 at every level (the plain Newton start).
__global__ __launch_bounds__(256) void k_broadcast(size_t ns, int nt, double* __restrict__ U,
                                                   const double* __restrict__ u0) {
  const size_t total = ns * (size_t)nt;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
    U[i] = u0[i % ns];
}

// ------------------------------------------------ coarse-grid initial iterate (Section 4)
// u^0 at the coarse nodes: the bilinear interpolant of the fine u^0. Coarse node k of an axis
// with n fine and nc coarse nodes lies at k n / nc (periodic) or (k + 1)(n + 1) / (nc + 1) - 1
// (Dirichlet interior nodes) fine spacings from fine node 0; the whole part and the remainder
// are taken in integers, so a coarse node that is a fine node (every node where the grids
// nest) takes that node's value unchanged. Dirichlet coarse nodes lie between fine nodes 0
// and n - 1, periodic ones wrap.
struct CfPos {
  int i0, i1;
  double t;  // weight of i1 (0: the node itself)
};
__device__ inline CfPos cf_pos(int k, int n, int nc, bool per) {
  const long num = per ? (long)k * n : (long)(k + 1) * (n + 1), den = per ? nc : nc + 1;
  CfPos q;
  q.i0 = (int)(num / den) - (per ? 0 : 1);
  const long r = num % den;
  q.t = (double)r / (double)den;
  q.i1 = r == 0 ? q.i0 : (per ? (q.i0 + 1) % n : q.i0 + 1);
  return q;
}
__global__ __launch_bounds__(256) void k_cf_sample(const double* __restrict__ u0, int nx, int ny, int nxc, int nyc,
                                                   int per, double* __restrict__ u0c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nxc * nyc) return;
  const CfPos px = cf_pos(i % nxc, nx, nxc, per), py = cf_pos(i / nxc, ny, nyc, per);
  auto row = [&](int y) {
    const double* r = u0 + (size_t)y * nx;
    return px.t == 0.0 ? r[px.i0] : (1.0 - px.t) * r[px.i0] + px.t * r[px.i1];
  };
  const double a = row(py.i0);
  u0c[i] = py.t == 0.0 ? a : (1.0 - py.t) * a + py.t * row(py.i1);
}

// Dirichlet data restricted to the coarse grid, for coarse levels m = 0..ntc-1 (fine level
// (m+1) cf - 1, layout south, north, west, east per level): the coarse problem's data bdc,
// its west and east parts as [m][yc] (the ends of the x lines), and the fine south and north
// rows of the same levels as [m][x] (the ends of the y lines).
__global__ __launch_bounds__(256) void k_cf_bdata(const double* __restrict__ bd, int nx, int ny, int nxc, int nyc,
                                                  int cf, int ntc, double* __restrict__ bdc,
                                                  double* __restrict__ west_c, double* __restrict__ east_c,
                                                  double* __restrict__ south_f, double* __restrict__ north_f) {
  const int nbc = 2 * (nxc + nyc), nbf = 2 * (nx + ny);
  const int per_level = nbc + 2 * nx;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ntc * per_level) return;
  const int m = t / per_level, k = t % per_level;
  const double* b = bd + (size_t)((m + 1) * cf - 1) * nbf;
  if (k < nbc) {
    double v;
    if (k < nxc) {
      v = b[(k + 1) * cf - 1];
    } else if (k < 2 * nxc) {
      v = b[nx + (k - nxc + 1) * cf - 1];
    } else if (k < 2 * nxc + nyc) {
      v = b[2 * nx + (k - 2 * nxc + 1) * cf - 1];
      west_c[m * nyc + (k - 2 * nxc)] = v;
    } else {
      v = b[2 * nx + ny + (k - 2 * nxc - nyc + 1) * cf - 1];
      east_c[m * nyc + (k - 2 * nxc - nyc)] = v;
    }
    bdc[(size_t)m * nbc + k] = v;
  } else if (k < nbc + nx) {
    south_f[(size_t)m * nx + (k - nbc)] = b[k - nbc];
  } else {
    north_f[(size_t)m * nx + (k - nbc - nx)] = b[nx + (k - nbc - nx)];
  }
}

// One 1-D interpolation pass: out[a][i][b] = sum_k W[i][k] v_k[a][b] over the nc nodes of
// the axis, v_k = in[a][k][b], or with in0 given v_0 = in0[b] and v_k = in[a][k - 1][b]; with
// edge values given (Dirichlet lines) also + Wlo[i] elo[a][b] + Whi[i] ehi[a][b]. Strides in
// elements; one thread per output, b fastest (threads of a wave then share i and read the
// weight row as uniform values).
__global__ __launch_bounds__(256) void k_interp_axis(const double* __restrict__ W, int nf, int nc,
                                                     const double* __restrict__ in, long isa, long isk, long isb,
                                                     const double* __restrict__ in0, double* __restrict__ out,
                                                     long osa, long osi, long osb, long na, long nb,
                                                     const double* __restrict__ Wlo, const double* __restrict__ Whi,
                                                     const double* __restrict__ elo, const double* __restrict__ ehi,
                                                     long esa, long esb) {
  const long total = na * nf * nb;
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long b = t % nb, r = t / nb;
    const int i = (int)(r % nf);
    const long a = r / nf;
    const double* w = W + (size_t)i * nc;
    const int k0 = in0 ? 1 : 0;
    double acc = in0 ? w[0] * in0[b] : 0.0;
    const long base = a * isa + b * isb;
    for (int k = k0; k < nc; ++k) acc = fma(w[k], in[base + (long)(k - k0) * isk], acc);
    if (elo) {
      const long e = a * esa + b * esb;
      acc = fma(Wlo[i], elo[e], acc);
      acc = fma(Whi[i], ehi[e], acc);
    }
    out[a * osa + (long)i * osi + b * osb] = acc;
  }
}

// Second derivatives of the not-a-knot spline in time at every node b (one thread each): nodes
// y_0 = in0[b], y_z = in[(z - 1) ns + b], z < N. The inner rows M_{z-1} + 4 M_z + M_{z+1} =
// 6 (y_{z-1} - 2 y_z + y_{z+1}) with the first and last rows reduced to 6 M_1 = d_1 and
// 6 M_{N-2} = d_{N-2} are solved by the Thomas algorithm (th[0..n): the eliminated
// super-diagonal, th[n..2n): the reciprocal pivots, n = N - 2; dp staged in M), then
// M_0 = 2 M_1 - M_2 and M_{N-1} = 2 M_{N-2} - M_{N-3}. N = 3 is one parabola, N = 2 a line.
__global__ __launch_bounds__(256) void k_spline_m_time(const double* __restrict__ th, int N,
                                                       const double* __restrict__ in0, const double* __restrict__ in,
                                                       long ns, double* __restrict__ M) {
  for (long b = (long)blockIdx.x * 256 + threadIdx.x; b < ns; b += (long)gridDim.x * 256) {
    auto y = [&](int z) -> double { return z == 0 ? in0[b] : in[(long)(z - 1) * ns + b]; };
    if (N < 3) {
      for (int z = 0; z < N; ++z) M[(long)z * ns + b] = 0.0;
      continue;
    }
    if (N == 3) {
      const double m = y(0) - 2.0 * y(1) + y(2);
      for (int z = 0; z < 3; ++z) M[(long)z * ns + b] = m;
      continue;
    }
    const int n = N - 2;
    double ym = y(0), y0 = y(1), dpp = 0.0;
    for (int i = 0; i < n; ++i) {
      const double yp = y(i + 2);
      const double d = 6.0 * (ym - 2.0 * y0 + yp);
      const double sub = (i == 0 || i == n - 1) ? 0.0 : 1.0;
      const double dp = (d - sub * dpp) * th[n + i];
      M[(long)(i + 1) * ns + b] = dp;
      dpp = dp;
      ym = y0;
      y0 = yp;
    }
    double mnext = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double m = M[(long)(i + 1) * ns + b] - (i + 1 < n ? th[i] * mnext : 0.0);
      M[(long)(i + 1) * ns + b] = m;
      mnext = m;
    }
    M[b] = 2.0 * M[ns + b] - M[2 * ns + b];
    M[(long)(N - 1) * ns + b] = 2.0 * M[(long)(N - 2) * ns + b] - M[(long)(N - 3) * ns + b];
  }
}

// The same not-a-knot second derivatives along the lines of a Dirichlet axis (one thread per
// line (a, b)): node 0 is the low edge value elo[a esa + b esb], node N - 1 the high one (zero
// when NULL), nodes 1..N-2 in[a isa + (z - 1) isk + b isb]; M[a osa + z osi + b osb]. In place
// of a dense N x N weight product per line, 4N operations.
__global__ __launch_bounds__(256) void k_spline_m_line(const double* __restrict__ th, int N,
                                                       const double* __restrict__ in, long isa, long isk, long isb,
                                                       const double* __restrict__ elo, const double* __restrict__ ehi,
                                                       long esa, long esb, double* __restrict__ M, long osa, long osi,
                                                       long osb, long na, long nb) {
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < na * nb; t += (long)gridDim.x * 256) {
    const long a = t / nb, b = t % nb, e = a * esa + b * esb, ib = a * isa + b * isb;
    double* __restrict__ m = M + a * osa + b * osb;
    auto y = [&](int z) -> double {
      if (z == 0) return elo ? elo[e] : 0.0;
      if (z == N - 1) return ehi ? ehi[e] : 0.0;
      return in[ib + (long)(z - 1) * isk];
    };
    if (N < 3) {
      for (int z = 0; z < N; ++z) m[(long)z * osi] = 0.0;
      continue;
    }
    if (N == 3) {
      const double c = y(0) - 2.0 * y(1) + y(2);
      for (int z = 0; z < 3; ++z) m[(long)z * osi] = c;
      continue;
    }
    const int n = N - 2;
    double ym = y(0), y0 = y(1), dpp = 0.0;
    for (int i = 0; i < n; ++i) {
      const double yp = y(i + 2);
      const double d = 6.0 * (ym - 2.0 * y0 + yp);
      const double sub = (i == 0 || i == n - 1) ? 0.0 : 1.0;
      const double dp = (d - sub * dpp) * th[n + i];
      m[(long)(i + 1) * osi] = dp;
      dpp = dp;
      ym = y0;
      y0 = yp;
    }
    double mnext = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double v = m[(long)(i + 1) * osi] - (i + 1 < n ? th[i] * mnext : 0.0);
      m[(long)(i + 1) * osi] = v;
      mnext = v;
    }
    m[0] = 2.0 * m[osi] - m[2 * osi];
    m[(long)(N - 1) * osi] = 2.0 * m[(long)(N - 2) * osi] - m[(long)(N - 3) * osi];
  }
}

// Evaluation of 1-D cubic splines from node values and second derivatives: fine point i lies
// in the interval (z0, z1) = zz[i] of the N spline nodes, and out[a][i][b] = w.x y(z0) + w.y
// y(z1) + w.z M(z0) + w.w M(z1) (w = wt[i]). Node z holds, with edges set, the edge values
// elo / ehi (zero when NULL) at z = 0 and z = N - 1; with in0 given, in0[b] at z = 0; else
// in[a][z - zoff][b]. M is [a][z][b] with strides msa, msk, msb.
__global__ __launch_bounds__(256) void k_spline_eval(const int2* __restrict__ zz, const double4* __restrict__ wt,
                                                     int nf, int N, int edges, const double* __restrict__ in,
                                                     long isa, long isk, long isb, int zoff,
                                                     const double* __restrict__ in0, const double* __restrict__ elo,
                                                     const double* __restrict__ ehi, long esa, long esb,
                                                     const double* __restrict__ M, long msa, long msk, long msb,
                                                     double* __restrict__ out, long osa, long osi, long osb, long na,
                                                     long nb) {
  const long total = na * nf * nb;
  auto point = [&](long a, int i, long b) {
    const int2 z = zz[i];
    const double4 w = wt[i];
    auto node = [&](int k) -> double {
      if (edges && (k == 0 || k == N - 1)) {
        const double* e = k == 0 ? elo : ehi;
        return e ? e[a * esa + b * esb] : 0.0;
      }
      if (in0 && k == 0) return in0[b];
      return in[a * isa + (long)(k - zoff) * isk + b * isb];
    };
    const double* m = M + a * msa + b * msb;
    double v = w.x * node(z.x);
    v = fma(w.y, node(z.y), v);
    v = fma(w.z, m[(long)z.x * msk], v);
    v = fma(w.w, m[(long)z.y * msk], v);
    out[a * osa + (long)i * osi + b * osb] = v;
  };
  if (total < (1L << 31)) {  // 32-bit index arithmetic (t + stride stays below 2^32)
    const unsigned nb32 = (unsigned)nb, nf32 = (unsigned)nf;
    for (unsigned t = blockIdx.x * 256u + threadIdx.x; t < (unsigned)total; t += gridDim.x * 256u) {
      const unsigned b = t % nb32, r = t / nb32;
      point((long)(r / nf32), (int)(r % nf32), (long)b);
    }
    return;
  }
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long b = t % nb, r = t / nb;
    point(r / nf, (int)(r % nf), b);
  }
}

// The time pass of the evaluation: one thread per node b and run of `run` fine levels
// (blockIdx.y), walking its levels in order; the two spline nodes of the current interval and
// their second derivatives stay in registers and are read again only when the interval changes
// (where the general kernel reads four values per fine level). Node 0 is in0[b] (u^0), node
// z > 0 is in[(z - 1) ns + b]; M is [z][ns]; out[i ns + b] for fine level i.
constexpr int kSplineRun = 16;  // fine levels per thread (more where gridDim.y would exceed 65535)
__global__ __launch_bounds__(256) void k_spline_eval_time(const int2* __restrict__ zz, const double4* __restrict__ wt,
                                                          int nf, int run, const double* __restrict__ in0,
                                                          const double* __restrict__ in, long ns,
                                                          const double* __restrict__ M, double* __restrict__ out) {
  const int i0 = blockIdx.y * run, i1 = min(nf, i0 + run);
  for (long b = (long)blockIdx.x * 256 + threadIdx.x; b < ns; b += (long)gridDim.x * 256) {
    auto y = [&](int z) -> double { return z == 0 ? in0[b] : in[(long)(z - 1) * ns + b]; };
    int cur = -1;
    double y0 = 0.0, y1 = 0.0, m0 = 0.0, m1 = 0.0;
    for (int i = i0; i < i1; ++i) {
      const int2 z = zz[i];
      if (z.x != cur) {
        cur = z.x;
        y0 = y(z.x);
        y1 = y(z.y);
        m0 = M[(long)z.x * ns + b];
        m1 = M[(long)z.y * ns + b];
      }
      const double4 w = wt[i];
      double v = w.x * y0;
      v = fma(w.y, y1, v);
      v = fma(w.z, m0, v);
      v = fma(w.w, m1, v);
      out[(long)i * ns + b] = v;
    }
  }
}

// Fill a small array of 64-bit words with zero (used instead of a memset node so that
// the sequence can be captured in a HIP graph).
__global__ void k_zero(unsigned long long* __restrict__ a, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) a[i] = 0ull;
}

}  // namespace pts
