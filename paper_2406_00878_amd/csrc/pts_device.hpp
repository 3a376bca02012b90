// Device-side building blocks of the space-time BDF1 kernels (gfx950).
//
// Discretization (Section 2, Eq. (3)), tau-scaled as in Section 3, Eq. (5):
//   G_P = u_P - u_P^{prev} + tau F_P,
//   F_P = cflux[(u_E^2 - u_W^2)/(2hx) + (u_N^2 - u_S^2)/(2hy)]
//         - [mu_e(u_E - u_P) - mu_w(u_P - u_W)]/hx^2 - [mu_n(u_N - u_P) - mu_s(u_P - u_S)]/hy^2
// with face viscosity mu_e = mu((u_P + u_E)/2), mu(v) = mu_a + mu_b v^2.
// Newton block A = I + tau dF/du (Eq. (6)); d mu_e / d u_P = d mu_e / d u_E = mu_b (u_P + u_E)/2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pts {

constexpr int kWave = 64;

// Problem scalars as the kernels see them (passed by value).
struct KProb {
  int nx, ny, nt, bc;  // bc: 0 Dirichlet, 1 periodic
  double dt, mu_a, mu_b, cf;
  double ihx, ihy, ihx2, ihy2;  // 1/hx, 1/hy, 1/hx^2, 1/hy^2
  const double* bdata;          // [nt][2(nx+ny)] or nullptr
  // constant-viscosity form: F = cx (E^2 - W^2) + cy (N^2 - S^2) - vx (E - 2P + W)
  // - vy (N - 2P + S); row of A: C = c0, W = -ax - bx u_W, E = -ax + bx u_E, S = -ay - by u_S,
  // N = -ay + by u_N (cx = cf / 2hx, vx = mu_a / hx^2, ax = tau vx, bx = tau cf / hx, c0 =
  // 1 + 2 (ax + ay), vp = 2 (vx + vy))
  double cx, cy, vx, vy, ax, ay, bx, by, c0, ic0, vp;  // ic0 = 1 / c0
  double axs, ays, bxs, bys;  // ax, ay, bx, by times 1 / c0: the rows of D^{-1} A
  const double* dts;          // [nt] step sizes tau_n (Eq. (3)), or nullptr: dt on every level
};

// The step-dependent constants of the constant-viscosity form, from k.dt.
__host__ __device__ inline void fold_tau(KProb& k) {
  k.ax = k.dt * k.vx;
  k.ay = k.dt * k.vy;
  k.bx = k.dt * k.cf * k.ihx;
  k.by = k.dt * k.cf * k.ihy;
  k.c0 = 1.0 + 2.0 * (k.ax + k.ay);
  k.ic0 = 1.0 / k.c0;
  k.axs = k.ax * k.ic0;
  k.ays = k.ay * k.ic0;
  k.bxs = k.bx * k.ic0;
  k.bys = k.by * k.ic0;
}

// The problem as level n (0-based) sees it: its own step tau_n when the steps vary.
__device__ __forceinline__ KProb at_level(const KProb& p, int n) {
  if (!p.dts) return p;
  KProb q = p;
  q.dt = p.dts[n];
  fold_tau(q);
  return q;
}

// Tiling of a level for the register-resident solve: a 64 x 64 region per work-group,
// of which the central TX x TY tile is written.
struct Geo {
  int TX, TY;  // tile edge
  int H;       // halo depth (neighbour exchanges one launch may perform)
  int tilesx;  // tiles along x
  int whole;   // 1: one region covers the whole Dirichlet domain (no halo needed)
};

// Work-groups go to the chip's 8 XCDs round-robin by linear id, and each XCD has an L2 of its
// own. xcd_band(b, n) renumbers index b of n (n a multiple of 8, else unchanged) so that each
// XCD receives one contiguous band of n/8 indices: tiles that share halo data then share an L2.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_band(unsigned b, unsigned n) {
  return n % kXcds ? b : (b % kXcds) * (n / kXcds) + b / kXcds;
}

struct Nb {
  double P, W, E, S, N;
};

// Element i of a level array through a 32-bit byte offset from the (wave-uniform) level
// base, which lets the loads and stores use scalar base + vector offset addressing.
// Levels hold at most 2^28 nodes, so the offset cannot wrap.
__device__ __forceinline__ double ld(const double* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (i << 3));
}
__device__ __forceinline__ void st(double* __restrict__ base, unsigned i, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (i << 3)) = v;
}

__device__ __forceinline__ double mu_of(const KProb& p, double v) { return p.mu_a + p.mu_b * v * v; }

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Value of level field `un` at (gx, gy) where (gx, gy) may be one node outside the
// domain: periodic wrap, or the level's Dirichlet data (zero if none).
__device__ __forceinline__ double node_value(const KProb& p, const double* __restrict__ un,
                                             const double* __restrict__ bd, int gx, int gy) {
  if (p.bc == 1) return un[(size_t)wrap(gy, p.ny) * p.nx + wrap(gx, p.nx)];
  if (gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny) return un[(size_t)gy * p.nx + gx];
  if (bd == nullptr) return 0.0;
  if (gy < 0) return bd[gx];
  if (gy >= p.ny) return bd[p.nx + gx];
  if (gx < 0) return bd[2 * p.nx + gy];
  return bd[2 * p.nx + p.ny + gy];
}

// Neighbours of the in-domain node (x, y). BC = 1: periodic indices wrap by one step
// (no integer division); BC = 0: Dirichlet neighbours outside the domain read the data.
template <int BC>
__device__ __forceinline__ Nb gather(const KProb& p, const double* __restrict__ un,
                                     const double* __restrict__ bd, int x, int y) {
  Nb u;
  const unsigned row = (unsigned)y * (unsigned)p.nx;
  u.P = ld(un, row + x);
  if (BC == 1) {
    const int xw = x == 0 ? p.nx - 1 : x - 1, xe = x == p.nx - 1 ? 0 : x + 1;
    const int ys = y == 0 ? p.ny - 1 : y - 1, yn = y == p.ny - 1 ? 0 : y + 1;
    u.W = ld(un, row + xw);
    u.E = ld(un, row + xe);
    u.S = ld(un, (unsigned)ys * (unsigned)p.nx + x);
    u.N = ld(un, (unsigned)yn * (unsigned)p.nx + x);
  } else {
    u.W = node_value(p, un, bd, x - 1, y);
    u.E = node_value(p, un, bd, x + 1, y);
    u.S = node_value(p, un, bd, x, y - 1);
    u.N = node_value(p, un, bd, x, y + 1);
  }
  return u;
}

__device__ __forceinline__ Nb gather(const KProb& p, const double* __restrict__ un,
                                     const double* __restrict__ bd, int x, int y) {
  return p.bc == 1 ? gather<1>(p, un, bd, x, y) : gather<0>(p, un, bd, x, y);
}

// Row of A = I + tau dF/du at node (x, y): C (self), W, E, S, N. Dirichlet boundary
// neighbours are data, so their entries are zero.
struct Row5 {
  double C, W, E, S, N;
};

// Forms of the flux that fix terms at compile time: general; constant viscosity (mu_b = 0,
// the viscous Burgers equation: coefficients folded into constants, E^2 - W^2 formed as
// (E - W)(E + W)); no convection (cf = 0, the heat equation: the convective terms, exact
// zeros there, are dropped). On its problems a special form agrees with the general form up
// to rounding.
enum { kFormGeneral = 0, kFormConstVisc = 1, kFormNoConv = 2 };

// F_P of Eq. (3) and the row of A at P from one evaluation of the face viscosities.
template <int BC, int FORM = kFormGeneral>
__device__ __forceinline__ double eval_point(const KProb& p, const Nb& u, int x, int y, Row5& r) {
  if constexpr (FORM == kFormConstVisc) {
    // the same discrete operator with the constant coefficients folded on the host, grouped
    // as F = (E + W)(cx (E - W) - vx) + (N + S)(cy (N - S) - vy) + vp P (nine operations)
    const double sx = u.E + u.W, sy = u.N + u.S;
    const double fx = sx * fma(p.cx, u.E - u.W, -p.vx);
    const double F = fma(p.vp, u.P, fma(sy, fma(p.cy, u.N - u.S, -p.vy), fx));
    r.C = p.c0;
    r.W = fma(-p.bx, u.W, -p.ax);
    r.E = fma(p.bx, u.E, -p.ax);
    r.S = fma(-p.by, u.S, -p.ay);
    r.N = fma(p.by, u.N, -p.ay);
    if (BC == 0) {
      if (x == 0) r.W = 0.0;
      if (x == p.nx - 1) r.E = 0.0;
      if (y == 0) r.S = 0.0;
      if (y == p.ny - 1) r.N = 0.0;
    }
    return F;
  }
  constexpr bool var_visc = FORM != kFormConstVisc, has_conv = FORM != kFormNoConv;
  const double me = var_visc ? mu_of(p, 0.5 * (u.P + u.E)) : p.mu_a;
  const double mw = var_visc ? mu_of(p, 0.5 * (u.P + u.W)) : p.mu_a;
  const double mn = var_visc ? mu_of(p, 0.5 * (u.P + u.N)) : p.mu_a;
  const double ms = var_visc ? mu_of(p, 0.5 * (u.P + u.S)) : p.mu_a;
  const double E2 = u.E * u.E, W2 = u.W * u.W, N2 = u.N * u.N, S2 = u.S * u.S, P2 = u.P * u.P;
  const double conv = has_conv ? p.cf * (0.5 * p.ihx * (E2 - W2) + 0.5 * p.ihy * (N2 - S2)) : 0.0;
  const double visc = p.ihx2 * (me * (u.E - u.P) - mw * (u.P - u.W)) + p.ihy2 * (mn * (u.N - u.P) - ms * (u.P - u.S));
  // d mu_face / d u_node = mu_b (u_P + u_X) / 2 for either node of the face
  const double hb = 0.5 * p.mu_b;
  const double qe = var_visc ? hb * (E2 - P2) : 0.0, qw = var_visc ? hb * (P2 - W2) : 0.0;
  const double qn = var_visc ? hb * (N2 - P2) : 0.0, qs = var_visc ? hb * (P2 - S2) : 0.0;
  const double cw = has_conv ? p.cf * u.W * p.ihx : 0.0, ce = has_conv ? p.cf * u.E * p.ihx : 0.0;
  const double cs = has_conv ? p.cf * u.S * p.ihy : 0.0, cn = has_conv ? p.cf * u.N * p.ihy : 0.0;
  r.C = 1.0 + p.dt * ((me + mw - qe + qw) * p.ihx2 + (mn + ms - qn + qs) * p.ihy2);
  r.W = p.dt * (-(mw - qw) * p.ihx2 - cw);
  r.E = p.dt * (-(me + qe) * p.ihx2 + ce);
  r.S = p.dt * (-(ms - qs) * p.ihy2 - cs);
  r.N = p.dt * (-(mn + qn) * p.ihy2 + cn);
  if (BC == 0) {
    if (x == 0) r.W = 0.0;
    if (x == p.nx - 1) r.E = 0.0;
    if (y == 0) r.S = 0.0;
    if (y == p.ny - 1) r.N = 0.0;
  }
  return conv - visc;
}

// Gershgorin radius of row r of D^{-1} A (infinite when the diagonal is not positive).
__device__ __forceinline__ double gersh(const Row5& r) {
  double g = (fabs(r.W) + fabs(r.E) + fabs(r.S) + fabs(r.N)) / fabs(r.C);
  if (!(r.C > 0.0) || g != g) g = __longlong_as_double(0x7ff0000000000000ll);
  return g;
}
// The same with 1 / C known (the constant-viscosity form's diagonal is the constant c0).
__device__ __forceinline__ double gersh(const Row5& r, double inv_c) {
  double g = (fabs(r.W) + fabs(r.E) + fabs(r.S) + fabs(r.N)) * inv_c;
  if (!(r.C > 0.0) || g != g) g = __longlong_as_double(0x7ff0000000000000ll);
  return g;
}

// ---------------------------------------------------------------- lane shifts
// DPP wavefront shifts by one lane with zero fill (bound_ctrl): shr makes lane i
// receive lane i-1 (lane 0 gets 0), shl makes lane i receive lane i+1 (lane 63 gets 0).
__device__ __forceinline__ int dpp_shr1_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_shl1_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }

__device__ __forceinline__ float lane_from_left(float v) {
  return __builtin_bit_cast(float, dpp_shr1_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_from_right(float v) {
  return __builtin_bit_cast(float, dpp_shl1_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_from_left(double v) {
  int2 q = __builtin_bit_cast(int2, v);
  q.x = dpp_shr1_i(q.x);
  q.y = dpp_shr1_i(q.y);
  return __builtin_bit_cast(double, q);
}
__device__ __forceinline__ double lane_from_right(double v) {
  int2 q = __builtin_bit_cast(int2, v);
  q.x = dpp_shl1_i(q.x);
  q.y = dpp_shl1_i(q.y);
  return __builtin_bit_cast(double, q);
}

// ------------------------------------------------------------- reductions
// max that propagates NaN (fmax would drop it)
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(a, b);
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o, kWave));
  return v;
}
// max of two values that are >= 0 or a NaN with a clear sign bit, NaN winning: read as
// unsigned 64-bit integers, the bit patterns of such values are ordered like the values and
// the NaN patterns lie above +inf (one integer compare instead of a NaN test and fmax)
__device__ __forceinline__ double max_nn(double a, double b) {
  return (unsigned long long)__double_as_longlong(a) > (unsigned long long)__double_as_longlong(b) ? a : b;
}
// A 64-bit value moved between lanes by one DPP control (applied to both halves).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  int2 q = __builtin_bit_cast(int2, v);
  q.x = __builtin_amdgcn_mov_dpp(q.x, CTRL, 0xF, 0xF, false);
  q.y = __builtin_amdgcn_mov_dpp(q.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, q);
}
// max_nn over each row of 16 lanes, left in every lane of the row: lane ^ 1 and lane ^ 2
// (quad permutations), then the half-row mirror (i <-> 7 - i) joins the two quads of each
// half row and the row mirror (i <-> 15 - i) the two halves. All in registers, no LDS.
__device__ __forceinline__ double row_max_nn(double v) {
  v = max_nn(v, dpp64<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = max_nn(v, dpp64<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = max_nn(v, dpp64<0x141>(v));  // row_half_mirror
  v = max_nn(v, dpp64<0x140>(v));  // row_mirror
  return v;
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  int2 q = __builtin_bit_cast(int2, v);
  q.x = __builtin_amdgcn_readlane(q.x, lane);
  q.y = __builtin_amdgcn_readlane(q.y, lane);
  return __builtin_bit_cast(double, q);
}
// max_nn over the whole wave, as a wave-uniform value (the four rows' maxima read back)
__device__ __forceinline__ double wave_max_nn(double v) {
  v = row_max_nn(v);
  return max_nn(max_nn(lane_value(v, 0), lane_value(v, 16)), max_nn(lane_value(v, 32), lane_value(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Max of non-negative doubles (NaN propagates as the largest bit pattern).
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* slot, double v) {
  unsigned long long b = __double_as_longlong(v);
  if (v != v) b = 0x7ff8000000000000ull;
  atomicMax(slot, b);
}

}  // namespace pts
