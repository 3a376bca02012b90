// Host side of the C ABI declared in include/pts.h.
//
// One all-at-once Newton step (Section 3, Eq. (5)-(6)) is
//   k_residual   (all levels)      r^n = -G^n(U), Gershgorin radii of D^{-1} A_n
//   k_level_solve, n = 1..N_t      du^n = A_n^{-1} (r^n + du^{n-1})   (Eq. (7), one level
//                                  per window; the only sequential part of the step)
//   k_update     (all levels)      U += dU, sum of dU^2
// The bulk schedule replays that sequence as one HIP graph per Newton step and reads
// back two scalars per step (max |r| and the largest Gershgorin radius) to decide
// convergence and the inner sweep count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pts.h"
#include "../../include/pts_no.h"
#include "pts_kernels.hip"
#include "pts_band.hpp"
#include "pts_prod.hpp"

using namespace pts;

namespace {
thread_local std::string g_err = "no error";
}

namespace pts_internal {
void set_error(const char* msg) { g_err = msg; }
}  // namespace pts_internal

namespace {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(PTS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kUpdateBlocks = 1024;
constexpr int kHalo = 16;  // halo of the 64 x 64 register region: tile 32 x 32
constexpr int kMaxWaveHalo = 24;  // deepest halo of a wavefront plan: tile edge >= 16

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int validate(const pts_problem* p) {
  if (!p) return fail(PTS_ERR_INVALID_ARG, "problem is NULL");
  if (p->kind != PTS_HEAT && p->kind != PTS_BURGERS) return fail(PTS_ERR_INVALID_ARG, "kind %d", p->kind);
  if (p->bc != PTS_DIRICHLET && p->bc != PTS_PERIODIC) return fail(PTS_ERR_INVALID_ARG, "bc %d", p->bc);
  if (p->nx < 1 || p->ny < 1 || p->nt < 1) return fail(PTS_ERR_INVALID_ARG, "sizes %d x %d x %d", p->nx, p->ny, p->nt);
  if ((long long)p->nx * p->ny > (1ll << 28)) return fail(PTS_ERR_INVALID_ARG, "level exceeds 2^28 nodes");
  if (p->nt > 65535) return fail(PTS_ERR_INVALID_ARG, "nt %d exceeds 65535", p->nt);
  if (p->precision != PTS_FP64 && p->precision != PTS_MIXED)
    return fail(PTS_ERR_INVALID_ARG, "precision %d", p->precision);
  if (!(p->hx > 0) || !(p->hy > 0) || !(p->dt > 0)) return fail(PTS_ERR_INVALID_ARG, "hx, hy, dt must be > 0");
  if (!(p->mu_a >= 0) || !(p->mu_b >= 0)) return fail(PTS_ERR_INVALID_ARG, "mu_a, mu_b must be >= 0");
  return PTS_OK;
}

KProb kprob(const pts_problem* p) {
  KProb k;
  k.nx = p->nx;
  k.ny = p->ny;
  k.nt = p->nt;
  k.bc = p->bc;
  k.dt = p->dt;
  k.mu_a = p->mu_a;
  k.mu_b = p->mu_b;
  k.cf = p->kind == PTS_BURGERS ? 0.5 : 0.0;
  k.ihx = 1.0 / p->hx;
  k.ihy = 1.0 / p->hy;
  k.ihx2 = k.ihx * k.ihx;
  k.ihy2 = k.ihy * k.ihy;
  k.bdata = p->bc == PTS_DIRICHLET ? p->bdata : nullptr;
  k.cx = 0.5 * k.cf * k.ihx;
  k.cy = 0.5 * k.cf * k.ihy;
  k.vx = k.mu_a * k.ihx2;
  k.vy = k.mu_a * k.ihy2;
  k.vp = 2.0 * (k.vx + k.vy);
  fold_tau(k);
  k.dts = p->dt_levels;
  return k;
}

// Workspace layout of one instance.
constexpr int kMaxStages = 16;  // Newton iterations overlapped by one wavefront sequence
constexpr int kMaxWindow = 64;  // longest Theorem-1 window

struct Layout {
  size_t R, dU, Xs, rho, scal, partial, rms, U1, rho_part, res_part, res_st, bar, u0copy, win, band, bstat, total;
};

// The banded direct level solve (pts_band.hpp) applies to Dirichlet problems of at most
// kBandMaxW nodes per direction; its factors take nt x nx ny x (2 nx + 1) doubles.
bool band_ok(const pts_problem* p) {
  return p->bc == PTS_DIRICHLET && p->nx <= kBandMaxW && p->ny <= kBandMaxW;
}

// Most tiles per level any wavefront plan uses: the deepest halo leaves 16 x 16 tiles (a
// small Dirichlet domain is one whole region).
size_t wave_tiles_max(const pts_problem* p) {
  if (p->bc == PTS_DIRICHLET && p->nx <= 64 && p->ny <= 64) return 1;
  const size_t e = 64 - 2 * kMaxWaveHalo;
  return ((p->nx + e - 1) / e) * ((p->ny + e - 1) / e);
}

Layout layout(const pts_problem* p) {
  const size_t ns = (size_t)p->nx * p->ny, st = ns * p->nt;
  Layout L;
  size_t o = 0;
  L.R = o;
  o = align_up(o + st * 8);
  L.dU = o;
  o = align_up(o + st * 8);
  L.Xs = o;
  o = align_up(o + ns * 8);
  L.rho = o;
  o = align_up(o + (size_t)p->nt * 16);
  L.scal = o;
  o = align_up(o + 4 * 8);
  L.partial = o;
  o = align_up(o + kUpdateBlocks * 8);
  L.rms = o;
  o = align_up(o + 8);
  L.U1 = o;  // second iterate slot of the wavefront schedule
  o = align_up(o + st * 8);
  {  // per-tile slots of the wavefront sequences, for the smallest tile any plan uses
    const size_t nt_max = wave_tiles_max(p);
    L.rho_part = o;
    o = align_up(o + (size_t)(kMaxStages + 1) * 4 * nt_max * 8);
    L.res_part = o;
    o = align_up(o + (size_t)(kMaxStages + 1) * nt_max * 8);
  }
  L.res_st = o;
  o = align_up(o + (kMaxStages + 1) * 8);
  L.bar = o;  // grid-barrier state of the cooperative wavefront sequence
  o = align_up(o + 8);
  L.u0copy = o;  // copy of u^0 for the wavefront sequences (keeps captured graphs independent of it)
  o = align_up(o + ns * 8);
  L.win = o;  // Theorem-1 windows: right-hand sides of a window plus two chain vectors
  o = align_up(o + (size_t)(std::min(kMaxWindow, p->nt) + 2) * ns * 8);
  L.band = o;  // banded LU factors of every level (band_ok problems only)
  o = align_up(o + (band_ok(p) ? st * (2 * (size_t)p->nx + 1) * 8 : 0));
  L.bstat = o;  // per-level zero-pivot flags of the factorisation
  o = align_up(o + (band_ok(p) ? (size_t)p->nt * 4 : 0));
  L.total = o;
  return L;
}

Geo geometry(const pts_problem* p, int halo = kHalo) {
  Geo g;
  if (p->bc == PTS_DIRICHLET && p->nx <= 64 && p->ny <= 64) {
    g.whole = 1;
    g.H = 0;
    g.TX = 64;
    g.TY = 64;
    g.tilesx = 1;
  } else {
    g.whole = 0;
    g.H = halo;
    g.TX = 64 - 2 * halo;
    g.TY = 64 - 2 * halo;
    g.tilesx = (p->nx + g.TX - 1) / g.TX;
  }
  return g;
}

int tiles(const pts_problem* p, const Geo& g) {
  if (g.whole) return 1;
  return g.tilesx * ((p->ny + g.TY - 1) / g.TY);
}

// Inner-solve plan: sweeps per pass and how passes are packed into launches.
// Passes per launch of a plan: at most kMaxPacks entries (a plan has at most 64 passes), held
// in place so that planning allocates nothing.
struct PackList {
  int v[kMaxPacks];
  int n = 0;
  void push_back(int x) {
    if (n < kMaxPacks) v[n++] = x;
  }
  size_t size() const { return (size_t)n; }
  int operator[](int i) const { return v[i]; }
  PackList& operator=(std::initializer_list<int> l) {
    n = 0;
    for (int x : l) push_back(x);
    return *this;
  }
};

struct Plan {
  int sweeps = 1;
  int passes = 1;   // total restarted passes per level
  PackList packs;   // passes per launch
  bool fp32 = false;
};

// Reduction factor of s Chebyshev sweeps on [1 - rho, 1 + rho]: 2 / T_s(1/rho).
double cheb_reduction(int s, double rho) {
  const double sigma = 1.0 / rho;
  return 2.0 / std::cosh(s * std::acosh(sigma));
}

Plan make_plan(const pts_problem* p, const pts_options* o, double rho_max, const Geo& g) {
  Plan pl;
  pl.fp32 = p->precision == PTS_MIXED;
  const double rho = std::min(std::max(rho_max, 1e-3), 0.999);
  double lin_tol = (o && o->lin_tol > 0) ? o->lin_tol : (pl.fp32 ? 1e-6 : 1e-9);
  // per-pass target: FP64 aims at lin_tol in one pass; FP32 passes stop near 1e-5
  const double pass_tol = pl.fp32 ? std::max(lin_tol, 1e-5) : lin_tol;
  int s = 1;
  if (o && o->sweeps > 0) {
    s = o->sweeps;
  } else {
    while (s < 4096 && cheb_reduction(s, rho) > pass_tol) ++s;
  }
  // One pass from zero needs s - 1 neighbour exchanges, a pass from an iterate s; the
  // halo bounds the exchanges of one launch.
  const bool fp32_fixed = pl.fp32 && o && o->refine > 0;
  // a pass runs at most kMaxSweeps - 1 sweeps (size of the kernel's weight table)
  s = std::min(s, kMaxSweeps - 1);
  bool one_pass = !fp32_fixed && (g.whole || s - 1 <= g.H) && cheb_reduction(s, rho) <= lin_tol;
  if (!g.whole && !one_pass) s = std::min(s, g.H);
  if (!g.whole && one_pass) s = std::min(s, g.H + 1);
  pl.sweeps = s;
  const double red = std::max(cheb_reduction(s, rho), pl.fp32 ? 1e-6 : 1e-15);
  int passes = 1;
  if (fp32_fixed) {
    passes = 1 + o->refine;
  } else if (!one_pass) {
    double r = red;
    while (r > lin_tol && passes < 64) {
      r *= red;
      ++passes;
    }
  }
  pl.passes = passes;
  // pack passes into launches: exchanges = (s - 1) for a pass from zero, s for a pass
  // that starts from an iterate
  int left = passes;
  bool first = true;
  while (left > 0) {
    int ex = 0, np = 0;
    while (left > 0) {
      const int need = first && np == 0 ? s - 1 : s;
      if (!g.whole && np > 0 && ex + need > g.H) break;
      ex += need;
      ++np;
      --left;
    }
    pl.packs.push_back(np);
    first = false;
  }
  return pl;
}


// Flux form of a problem (see eval_point): constant viscosity, no convection, or general.
int flux_form(const pts_problem* p) {
  if (p->mu_b == 0.0) return kFormConstVisc;
  if (p->kind == PTS_HEAT) return kFormNoConv;
  return kFormGeneral;
}

// Level solver for blocks whose Jacobi-scaled Gershgorin radius is rho: the register-resident
// Chebyshev iteration needs rho < 1 (a Gershgorin disc bounds the Jacobi spectrum) and a real
// spectrum; with a complex one (central convection at cell Peclet numbers above 2, flagged by
// cplx) Chebyshev on [-rho, rho] diverges once rho exceeds 1/sqrt(2). Returns 0 (Chebyshev),
// 1 (banded direct solve) or -1 (neither applies).
constexpr double kCplxRho = 0.7;
int level_solver(const pts_problem* p, double rho, bool cplx) {
  const bool cheb = rho < 1.0 && !(cplx && rho > kCplxRho);
  if (cheb) return 0;
  return band_ok(p) ? 1 : -1;
}

// The all-level residual kernel for a problem's boundary kind and flux form.
typedef void (*ResidualKernel)(KProb, const double*, const double*, double*, double*, unsigned long long*);
ResidualKernel residual_kernel(const pts_problem* p) {
  const bool per = p->bc == PTS_PERIODIC;
  switch (flux_form(p)) {
    case kFormConstVisc: return per ? k_residual<1, kFormConstVisc> : k_residual<0, kFormConstVisc>;
    case kFormNoConv: return per ? k_residual<1, kFormNoConv> : k_residual<0, kFormNoConv>;
    default: return per ? k_residual<1, kFormGeneral> : k_residual<0, kFormGeneral>;
  }
}

// lvl_bits: 2 words per level (max |r|, max radius), zeroed here; scal (nullable)
// receives the maxima over levels.
int launch_residual(const pts_problem* p, const KProb& kp, const double* U, const double* u0, double* R,
                    double* coef, unsigned long long* lvl_bits, unsigned long long* scal, hipStream_t s) {
  const int tilesx = (p->nx + 63) / 64, tilesy = (p->ny + kResRows - 1) / kResRows;
  if (lvl_bits) hipLaunchKernelGGL(k_zero, dim3((2 * p->nt + 255) / 256), dim3(256), 0, s, lvl_bits, 2 * p->nt);
  dim3 grid((unsigned)(tilesx * tilesy), (unsigned)p->nt);
  hipLaunchKernelGGL(residual_kernel(p), grid, dim3(256), 0, s, kp, U, u0, R, coef, lvl_bits);
  if (scal) hipLaunchKernelGGL(k_level_max, dim3(1), dim3(256), 0, s, lvl_bits, p->nt, scal);
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

// Eq. (7) by banded direct solves (Section 8): every level's block factorised in one launch,
// then the chain of substitutions in one work-group; a zero pivot is reported by the next
// status check (status words per level in the workspace).
int launch_band(const pts_problem* p, const KProb& kp, const double* U, const double* R, double* dU, double* B,
                int* bstat, hipStream_t s, int* launches) {
  auto fac = flux_form(p) == kFormConstVisc ? k_band_factor<kFormConstVisc>
             : (flux_form(p) == kFormNoConv ? k_band_factor<kFormNoConv> : k_band_factor<kFormGeneral>);
  hipLaunchKernelGGL(fac, dim3((unsigned)p->nt), dim3(256), 0, s, kp, U, B, bstat);
  hipLaunchKernelGGL(k_band_chain, dim3(1), dim3(64), 0, s, p->nx, p->ny, p->nt, (const double*)B, R, dU);
  *launches += 2;
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

// Forward block substitution over all levels: du^n = A_n^{-1}(r^n + du^{n-1}) (Eq. (7)).
struct Prof;
void prof_begin(Prof* pr, int kind, hipStream_t s);
void prof_end(Prof* pr, hipStream_t s, double bytes);
void prof_end_count(Prof* pr, hipStream_t s, double bytes, int count);  // interval covering `count` launches

int launch_chain(const pts_problem* p, const KProb& kp, const double* U, const double* R, double* dU, double* Xs,
                 const double* rho, const Plan& pl, const Geo& g, hipStream_t s, int* launches, Prof* pr) {
  const size_t ns = (size_t)p->nx * p->ny;
  const int nb = tiles(p, g);
  const int nl = (int)pl.packs.size();
  // profiling brackets the whole chain (per-launch events would add their own overhead)
  prof_begin(pr, 1, s);
  double bytes = 0.0;
  for (int n = 0; n < p->nt; ++n) {
    const double* prev = n == 0 ? nullptr : dU + (size_t)(n - 1) * ns;
    double* out = dU + (size_t)n * ns;
    // ping-pong between the scratch level and dU[n] so that the last launch writes dU[n]
    const double* xin = nullptr;
    for (int l = 0; l < nl; ++l) {
      double* xo = ((nl - 1 - l) % 2 == 0) ? out : Xs;
      const bool per = p->bc == PTS_PERIODIC;
      auto kern = pl.fp32 ? (per ? k_level_solve<float, 1> : k_level_solve<float, 0>)
                          : (per ? k_level_solve<double, 1> : k_level_solve<double, 0>);
      hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, s, kp, n, U, R + (size_t)n * ns, prev, xin, xo, rho,
                         g, pl.packs[l], pl.sweeps);
      bytes += 8.0 * (double)ns * (3 + (prev ? 1 : 0) + (xin ? 1 : 0));
      xin = xo;
      ++*launches;
    }
  }
  prof_end_count(pr, s, bytes, p->nt * nl);
  HIPCHK(hipGetLastError());
  return PTS_OK;
}


// Theorem 1 inside windows of W levels (Section 4, Eq. (8); recursion of Section 5):
// level w of the window [w0, w0+W) solves P_w du^w = rt^w with P_w = A_{w0} ... A_w,
// rt^{w0} = r^{w0} + du^{w0-1} (the -I block of Eq. (6) carried into the window) and
// rt^w = rt^{w-1} + A_{w0}(A_{w0+1}(... A_{w-1} r^w)). P_w is applied through its factors:
// du^w = A_w^{-1}(... A_{w0}^{-1} rt^w). Every window's levels are decoupled from each
// other; W = 1 is the block inverse of Eq. (7).
int launch_windows(const pts_problem* p, const KProb& kp, const double* U, const double* R, double* dU,
                   double* Xs, const double* rho, const Plan& pl, const Geo& g, int W, char* ws, const Layout& L,
                   hipStream_t s, int* launches) {
  const size_t ns = (size_t)p->nx * p->ny;
  const int nb = tiles(p, g);
  double* rt = (double*)(ws + L.win);
  double* t1 = rt + (size_t)std::min(kMaxWindow, p->nt) * ns;
  double* t2 = t1 + ns;
  const unsigned ablocks = (unsigned)((ns + 255) / 256);
  const unsigned cblocks = (unsigned)std::min<size_t>((ns + 255) / 256, 4096);
  const bool per = p->bc == PTS_PERIODIC;
  auto apply = per ? k_apply<1> : k_apply<0>;
  auto solve = pl.fp32 ? (per ? k_level_solve<float, 1> : k_level_solve<float, 0>)
                       : (per ? k_level_solve<double, 1> : k_level_solve<double, 0>);
  const int nl = (int)pl.packs.size();
  for (int w0 = 0; w0 < p->nt; w0 += W) {
    const int Wc = std::min(W, p->nt - w0);
    // rt^{w0}
    hipLaunchKernelGGL(k_add, dim3(cblocks), dim3(256), 0, s, ns, R + (size_t)w0 * ns,
                       w0 > 0 ? dU + (size_t)(w0 - 1) * ns : nullptr, rt);
    ++*launches;
    for (int k = 1; k < Wc; ++k) {
      // v = A_{w0} ... A_{w0+k-1} r^{w0+k}, innermost factor first
      const double* src = R + (size_t)(w0 + k) * ns;
      double* dst = t1;
      for (int m = w0 + k - 1; m >= w0; --m) {
        hipLaunchKernelGGL(apply, dim3(ablocks), dim3(256), 0, s, kp, m, U, src, dst);
        ++*launches;
        src = dst;
        dst = dst == t1 ? t2 : t1;
      }
      hipLaunchKernelGGL(k_add, dim3(cblocks), dim3(256), 0, s, ns, rt + (size_t)(k - 1) * ns, src,
                         rt + (size_t)k * ns);
      ++*launches;
    }
    for (int k = 0; k < Wc; ++k) {
      // du^{w0+k} = A_{w0+k}^{-1} ... A_{w0}^{-1} rt^{w0+k}
      const double* y = rt + (size_t)k * ns;
      for (int i = w0; i <= w0 + k; ++i) {
        double* out = i == w0 + k ? dU + (size_t)(w0 + k) * ns : (y == t1 ? t2 : t1);
        const double* xin = nullptr;
        for (int l = 0; l < nl; ++l) {
          // restarted passes ping-pong through the scratch level, the last one into `out`
          double* xo = ((nl - 1 - l) % 2 == 0) ? out : Xs;
          hipLaunchKernelGGL(solve, dim3(nb), dim3(kThreads), 0, s, kp, i, U, y, nullptr, xin, xo, rho, g,
                             pl.packs[l], pl.sweeps);
          ++*launches;
          xin = xo;
        }
        y = out;
      }
    }
  }
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

struct HostScalars {
  double* h = nullptr;  // pinned, 512 doubles: [0] max|r|, [1] rho_max, [2] sum dU^2, or the
                        // per-stage residuals of a wavefront sequence
  ~HostScalars() {
    if (h) (void)hipHostFree(h);
  }
};
thread_local HostScalars g_host;

int host_scalars(double** out) {
  if (!g_host.h) HIPCHK(hipHostMalloc((void**)&g_host.h, 4096, hipHostMallocDefault));
  *out = g_host.h;
  return PTS_OK;
}

// Scratch of pts_newton_step_static: a file-scope device array, one copy per GPU, held from
// the library's load on that GPU to the end of the process. The array's name is a host-side
// stand-in in host code: its device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is passed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

int static_scratch(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PTS_ERR_INVALID_ARG, "device %d beyond %d", dev, kMaxDevices);
  static std::mutex m;
  static void* addr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lk(m);
  if (!addr[dev]) {
    void* a = nullptr;
    HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    if (!a || (uintptr_t)a % kAlign) return fail(PTS_ERR_HIP, "static scratch has no usable device address");
    addr[dev] = a;
  }
  *out = addr[dev];
  return PTS_OK;
}

// Optional per-kernel timing with HIP events recorded on the launch stream.
struct Prof {
  struct Rec {
    int kind;  // 0..3: pts_stats.prof_ms classes; kKern + j: pts_stats.kern_ms[j]
    hipEvent_t a, b;
    int count;     // launches the interval covers
    double bytes;  // algorithmic bytes of those launches
  };
  static constexpr int kKern = 8;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;  // events of collected records, reused
  double bytes = 0.0;
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else {
      (void)hipEventCreate(&e);
    }
    return e;
  }
  void begin(int kind, hipStream_t s) {
    Rec r{kind, event(), event(), 1, 0.0};
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end(hipStream_t s) { (void)hipEventRecord(recs.back().b, s); }
  // add the recorded intervals to st (the stream must have reached them)
  void collect(pts_stats* st) {
    for (auto& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && st) {
        if (r.kind < kKern) {
          st->prof_ms[r.kind] += ms;
          st->prof_count[r.kind] += r.count;
        } else {
          st->kern_ms[r.kind - kKern] += ms;
          st->kern_count[r.kind - kKern] += r.count;
          st->kern_bytes[r.kind - kKern] += r.bytes;
        }
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
    if (st) st->level_solve_bytes = bytes;
  }
  ~Prof() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Device state of one instance bound to a caller workspace.
void prof_begin(Prof* pr, int kind, hipStream_t s) {
  if (pr) pr->begin(kind, s);
}
void prof_end(Prof* pr, hipStream_t s, double bytes) {
  if (pr) {
    pr->end(s);
    pr->bytes += bytes;
  }
}
void prof_end_count(Prof* pr, hipStream_t s, double bytes, int count) {
  if (pr) {
    prof_end(pr, s, bytes);
    pr->recs.back().count = count;
  }
}

struct Instance {
  Prof* prof = nullptr;
  const pts_problem* p = nullptr;
  KProb kp;
  Layout L;
  Geo g;
  double* R;
  double* dU;
  double* Xs;
  unsigned long long* rho;
  unsigned long long* scal;  // [0] max |r|, [1] rho_max
  double* partial;
  double* rms;

  void bind(const pts_problem* pp, void* w) {
    wsb = (char*)w;
    p = pp;
    kp = kprob(pp);
    L = layout(pp);
    g = geometry(pp);
    char* ws = (char*)w;
    R = (double*)(ws + L.R);
    dU = (double*)(ws + L.dU);
    Xs = (double*)(ws + L.Xs);
    rho = (unsigned long long*)(ws + L.rho);
    scal = (unsigned long long*)(ws + L.scal);
    partial = (double*)(ws + L.partial);
    rms = (double*)(ws + L.rms);
  }

  // residual at U with per-level and global maxima (fill kernels, so the sequence is
  // graph-safe)
  int residual(const double* U, const double* u0, hipStream_t s, int* launches, bool store_r = true) {
    *launches += 3;
    prof_begin(prof, 0, s);
    int rc = launch_residual(p, kp, U, u0, store_r ? R : nullptr, nullptr, rho, scal, s);
    if (prof) prof->end(s);
    return rc;
  }

  int window = 1;
  char* wsb = nullptr;
  bool band = false;  // level solves by banded LU (pts_band.hpp) instead of Chebyshev
  int bflag = 0;      // host copy of the zero-pivot flag of the last factorisation

  int step_body(double* U, const Plan& pl, hipStream_t s, int* launches) {
    int rc = PTS_OK;
    if (band) {
      int* bstat = (int*)(wsb + L.bstat);
      hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (unsigned long long*)bstat, 1);
      ++*launches;
      prof_begin(prof, 1, s);
      rc = launch_band(p, kp, U, R, dU, (double*)(wsb + L.band), bstat, s, launches);
      prof_end(prof, s, 0.0);
    } else {
      rc = window > 1 ? launch_windows(p, kp, U, R, dU, Xs, (const double*)rho, pl, g, window, wsb, L, s, launches)
                      : launch_chain(p, kp, U, R, dU, Xs, (const double*)rho, pl, g, s, launches, prof);
    }
    if (rc) return rc;
    const size_t count = (size_t)p->nx * p->ny * p->nt;
    prof_begin(prof, 2, s);
    hipLaunchKernelGGL(k_update, dim3(kUpdateBlocks), dim3(256), 0, s, count, U, dU, partial);
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, partial, kUpdateBlocks, rms);
    if (prof) prof->end(s);
    *launches += 2;
    HIPCHK(hipGetLastError());
    return PTS_OK;
  }

  int read_scalars(double* hs, bool with_rms, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(hs, scal, 16, hipMemcpyDeviceToHost, s));
    if (with_rms) HIPCHK(hipMemcpyAsync(hs + 2, rms, 8, hipMemcpyDeviceToHost, s));
    if (band) HIPCHK(hipMemcpyAsync(&bflag, wsb + L.bstat, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PTS_OK;
  }
};

int check_ws(const pts_problem* p, void* ws, size_t bytes) {
  if (!ws) return fail(PTS_ERR_WORKSPACE, "workspace is NULL");
  const size_t need = layout(p).total;
  if (bytes < need) return fail(PTS_ERR_WORKSPACE, "workspace %zu bytes < required %zu", bytes, need);
  if ((uintptr_t)ws % kAlign) return fail(PTS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return PTS_OK;
}

int check_opts(const pts_options* o) {
  if (!o) return PTS_OK;
  if (o->window > kMaxWindow) return fail(PTS_ERR_INVALID_ARG, "window %d exceeds %d", o->window, kMaxWindow);
  if (o->window > 1 && o->schedule == PTS_SCHED_PIPELINE)
    return fail(PTS_ERR_INVALID_ARG, "Theorem-1 windows run in the bulk schedule");
  if (o->window < 0 || o->sweeps < 0 || o->lin_tol < 0)
    return fail(PTS_ERR_INVALID_ARG, "negative option");
  if (o->refine >= kMaxPacks) return fail(PTS_ERR_INVALID_ARG, "refine %d exceeds %d", o->refine, kMaxPacks - 1);
  if (o->schedule != PTS_SCHED_AUTO && o->schedule != PTS_SCHED_BULK && o->schedule != PTS_SCHED_PIPELINE)
    return fail(PTS_ERR_INVALID_ARG, "schedule %d not available", o->schedule);
  if (o->stages < 0 || o->stages > kMaxStages) return fail(PTS_ERR_INVALID_ARG, "stages %d", o->stages);
  if (o->wave_launch != 0 && o->wave_launch != 1) return fail(PTS_ERR_INVALID_ARG, "wave_launch %d", o->wave_launch);
  if (o->barrier_spins < 0) return fail(PTS_ERR_INVALID_ARG, "negative option");
  return PTS_OK;
}

// Graph of one Newton step (chain + update + next residual), cached per plan.
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  int sweeps = -1, passes = -1;
  ~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

int capture_step(Instance& in, double* U, const double* u0, const Plan& pl, hipStream_t s, StepGraph& sg) {
  if (sg.exec) {
    HIPCHK(hipGraphExecDestroy(sg.exec));
    sg.exec = nullptr;
  }
  // Capture on a private stream (the caller's stream may be the null stream, which
  // cannot be captured); the executable graph is then launched on the caller's stream.
  static thread_local hipStream_t cap = nullptr;
  if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  (void)s;
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int dummy = 0;
  int rc = in.step_body(U, pl, cap, &dummy);
  if (!rc) rc = in.residual(U, u0, cap, &dummy);
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (rc) return rc;
  if (e != hipSuccess) return fail(PTS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(PTS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  sg.sweeps = pl.sweeps;
  sg.passes = pl.passes;
  return PTS_OK;
}

// Whether central convection may give the Jacobi iteration matrix complex eigenvalues: the
// off-diagonal pair of a row, -a - b u_W and -a + b u_E (a = tau mu / h^2, b = tau cflux / h),
// has entries of opposite sign once b |u| > a, i.e. at cell Peclet numbers |u| h / mu above
// 1 / cflux = 2. |u| is bounded by the data (max |u0|, max |bdata|, with a 5 % margin for
// overshoots of the discrete solution) and mu >= mu_a. Reads two scalars back (synchronises).
int convection_flag(const pts_problem* p, const double* u0, void* ws, hipStream_t s, double* hbuf, bool* cplx) {
  *cplx = false;
  if (p->kind != PTS_BURGERS) return PTS_OK;
  const Layout L = layout(p);
  unsigned long long* sc = (unsigned long long*)((char*)ws + L.scal) + 2;
  hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, u0, (size_t)p->nx * p->ny, sc);
  if (p->bdata)
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, p->bdata, (size_t)p->nt * 2 * (p->nx + p->ny), sc + 1);
  else
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, sc + 1, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hbuf, sc, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double umax = 1.05 * std::max(hbuf[0], hbuf[1]);
  const double h = std::max(p->hx, p->hy);
  *cplx = p->mu_a > 0 ? 0.5 * umax * h / p->mu_a > 1.0 : umax > 0.0;
  return PTS_OK;
}

// hs_caller: host buffer of 4 doubles for the scalars read back per step, or NULL for the
// thread's pinned buffer. cplx: see convection_flag.
int solve_bulk(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
               const pts_options* o, pts_stats* st, hipStream_t s, bool single_step, bool cplx,
               double* hs_caller = nullptr) {
  Instance in;
  in.bind(p, ws);
  in.window = (o && o->window > 1) ? std::min(o->window, std::min(kMaxWindow, p->nt)) : 1;
  Prof prof;
  const bool profiling = o && o->profile;
  if (profiling) in.prof = &prof;
  double* hs = hs_caller;
  int rc = hs ? PTS_OK : host_scalars(&hs);
  if (rc) return rc;
  const bool use_graph =
      !single_step && !profiling && (!o || o->use_graph != 0 || o->schedule == PTS_SCHED_AUTO);
  StepGraph sg;
  int launches = 0;
  rc = in.residual(U, u0, s, &launches);
  if (rc) return rc;
  rc = in.read_scalars(hs, false, s);
  if (rc) return rc;
  Plan pl;
  double planned_rho = -1.0;
  int it = 0;
  for (;;) {
    const double res = hs[0], rhom = hs[1];
    if (st && it < PTS_MAX_HIST) {
      st->res_inf[it] = res;
      st->rho_max[it] = rhom;
      if (it > 0) st->upd_rms[it] = std::sqrt(hs[2] / ((double)p->nx * p->ny * p->nt));
    }
    if (!std::isfinite(res) || !std::isfinite(rhom)) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_NONFINITE, "non-finite residual at Newton step %d", it);
    }
    if (!single_step && res <= tol) {
      if (st) {
        st->iterations = it;
        st->converged = 1;
        st->launches = launches;
      }
      if (profiling) prof.collect(st);
      return PTS_OK;
    }
    if (in.band && in.bflag) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_SINGULAR, "zero pivot in the banded LU of a level block at Newton step %d", it);
    }
    const int solver = level_solver(p, rhom, cplx);
    if (solver < 0) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_NOT_DOMINANT, "no convergent level solve: Gershgorin radius %.3g%s, and the banded LU "
                  "needs a Dirichlet grid of at most %d nodes per direction", rhom,
                  cplx ? " with cell Peclet numbers above 2" : "", kBandMaxW);
    }
    in.band = solver == 1;
    if ((single_step && it == 1) || (!single_step && it >= max_iter)) {
      if (st) {
        st->iterations = it;
        st->launches = launches;
      }
      if (profiling) prof.collect(st);
      if (single_step) return PTS_OK;
      return fail(PTS_ERR_NOT_CONVERGED, "not converged after %d Newton steps (|R| = %.3e)", it, res);
    }
    // plan the inner solves from the current largest Gershgorin radius (the graph is
    // re-captured only when the sweep or pass count changes)
    if (rhom != planned_rho) {
      planned_rho = rhom;
      pl = make_plan(p, o, std::min(planned_rho * 1.02, 0.999), in.g);
    }
    if (st) {
      st->sweeps = in.band ? 0 : pl.sweeps;
      st->refine = in.band ? 0 : pl.passes - 1;
      st->window = in.band ? 1 : in.window;
      st->schedule = PTS_SCHED_BULK;
    }
    if (use_graph && !in.band) {
      if (sg.sweeps != pl.sweeps || sg.passes != pl.passes) {
        rc = capture_step(in, U, u0, pl, s, sg);
        if (rc) return rc;
      }
      HIPCHK(hipGraphLaunch(sg.exec, s));
      ++launches;
    } else {
      rc = in.step_body(U, pl, s, &launches);
      if (rc) return rc;
      rc = in.residual(U, u0, s, &launches);
      if (rc) return rc;
    }
    ++it;
    rc = in.read_scalars(hs, true, s);
    if (rc) return rc;
  }
}


// ------------------------------------------------------------ wavefront schedule
// Inner-solve plan for the wavefront kernel. Every pass of a level runs in the one launch
// and the tile must stay valid one node beyond its edge, so the halo is the number of
// neighbour exchanges plus one: H = (s - 1) + (P - 1) s + 1, tile edge 64 - 2H. Fewer
// sweeps therefore also mean larger tiles and fewer work-groups per level.

int wave_halo(const Plan& pl) { return (pl.sweeps - 1) + (pl.passes - 1) * pl.sweeps + 1; }

// Work of one (stage, level) in region-sweeps: tiles x sweeps x passes.
double wave_cost(const pts_problem* p, const Plan& pl) {
  const Geo g = geometry(p, wave_halo(pl));
  return (double)tiles(p, g) * pl.sweeps * pl.passes;
}

// Cheapest plan whose reduction reaches lin_tol (explicit sweeps/refine options are obeyed).
bool make_wave_plan(const pts_problem* p, const pts_options* o, double rho_max, double lin_tol, Plan* out) {
  const bool fp32 = p->precision == PTS_MIXED;
  const bool whole = geometry(p).whole;
  const double rho = std::min(std::max(rho_max, 1e-3), 0.999);
  const double floor_red = fp32 ? 1e-6 : 1e-15;
  Plan best;
  double best_cost = 0.0, best_red = 1.0;
  bool found = false;
  for (int s = 1; s < kMaxSweeps; ++s) {
    if (o && o->sweeps > 0 && s != o->sweeps) continue;
    for (int P = 1; P <= 8; ++P) {
      if (!fp32 && P > 1) break;  // FP64 passes are one long Chebyshev run
      if (fp32 && o && o->refine >= 0 && !(o->refine == 0 && o->sweeps == 0) && P != 1 + o->refine) continue;
      Plan pl;
      pl.fp32 = fp32;
      pl.sweeps = s;
      pl.passes = P;
      pl.packs = {P};
      if (!whole && wave_halo(pl) > kMaxWaveHalo) continue;
      const double red = std::pow(std::max(cheb_reduction(s, rho), floor_red), P);
      const double cost = whole ? (double)s * P : wave_cost(p, pl);
      const bool ok = red <= lin_tol;
      const bool best_ok = found && best_red <= lin_tol;
      if (!found || (ok && !best_ok) || (ok && best_ok && cost < best_cost) || (!ok && !best_ok && red < best_red)) {
        best = pl;
        best_cost = cost;
        best_red = red;
        found = true;
      }
    }
  }
  if (!found) return false;
  *out = best;
  return best_red <= 1e-2;
}

// Autotuned choices per problem signature and tolerance: inner sweeps and passes of the
// wavefront kernel and the Newton steps they needed.
// Entries for one instance and for batches of instances of the problem (batch = 1) are kept
// apart: a batch's launches are throughput-bound, one instance's latency-bound, and the
// fastest plans differ.
struct StageCache {
  struct E {
    int nx, ny, nt, kind, bc, prec, tag, batch;
    double dt, mu_a, mu_b, tol;
    int sweeps, passes, steps;
  };
  std::vector<E> v;
  E* find(const pts_problem* p, double tol, int tag, int batch = 0) {
    for (auto& e : v)
      if (e.nx == p->nx && e.ny == p->ny && e.nt == p->nt && e.kind == p->kind && e.bc == p->bc &&
          e.prec == p->precision && e.tag == tag && e.batch == batch && e.dt == p->dt && e.mu_a == p->mu_a &&
          e.mu_b == p->mu_b && e.tol == tol)
        return &e;
    return nullptr;
  }
  // keep_max: the entry keeps the largest step count seen with this plan. A sequence with a
  // spare stage costs two more diagonal launches, one stage short costs a second sequence.
  void put(const pts_problem* p, double tol, int tag, int sweeps, int passes, int steps, bool keep_max = false,
           int batch = 0) {
    if (E* e = find(p, tol, tag, batch)) {
      if (keep_max && e->sweeps == sweeps && e->passes == passes) steps = std::max(steps, e->steps);
      e->sweeps = sweeps;
      e->passes = passes;
      e->steps = steps;
      return;
    }
    if (v.size() > 64) v.clear();
    v.push_back({p->nx, p->ny, p->nt, p->kind, p->bc, p->precision, tag, batch, p->dt, p->mu_a, p->mu_b, tol,
                 sweeps, passes, steps});
  }
};
thread_local StageCache g_stage_cache;
int ctag(const pts_options* o) { return o ? o->cache_tag : 0; }

// Inner plan and stage count of the next wavefront sequence after `it` Newton steps: explicit
// options, else the cached entry (ce, may be NULL), else the cheapest plan that reaches lin_tol
// (default 1e-4: the wavefront runs inexact Newton steps) for the radius rho. K: options, else
// the steps the cached entry still expects, else 4; at most max_iter - it. False when no plan
// reaches the reduction.
bool next_wave_plan(const pts_problem* p, const pts_options* o, const StageCache::E* ce, double rho, int it,
                    int max_iter, Plan* pl, int* K) {
  const double lin_tol = (o && o->lin_tol > 0) ? o->lin_tol : 1e-4;
  const bool explicit_inner = o && (o->sweeps > 0 || o->refine > 0 || o->lin_tol > 0);
  if (ce && !explicit_inner && ce->sweeps > 0) {
    pl->fp32 = p->precision == PTS_MIXED;
    pl->sweeps = ce->sweeps;
    pl->passes = ce->passes;
    pl->packs = {pl->passes};
  } else if (!make_wave_plan(p, o, std::min(rho * 1.02, 0.999), lin_tol, pl)) {
    return false;
  }
  int k = (o && o->stages > 0) ? o->stages : (ce && ce->steps > it ? ce->steps - it : 4);
  *K = std::max(1, std::min(std::min(k, kMaxStages), max_iter - it));
  return true;
}

// Executable graph of one wavefront sequence, reused while the launch arguments match.
struct WaveGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;
};
thread_local std::vector<WaveGraph> g_wave_graphs;


// The wavefront kernel for a problem (inner type, boundary kind, flux form): one launch per
// anti-diagonal, or with seq the cooperative whole-sequence form.
typedef void (*WaveKernel)(KProb, WaveArgs, Geo, int, int, int);
typedef void (*WaveSeqKernel)(KProb, WaveArgs, Geo, int, int, int, unsigned*, unsigned);
template <typename T, int BC>
const void* wave_kernel_bc(int form, bool seq) {
  if (seq)
    return (const void*)(form == kFormConstVisc ? (WaveSeqKernel)k_level_wave_seq<T, BC, kFormConstVisc>
                         : form == kFormNoConv  ? (WaveSeqKernel)k_level_wave_seq<T, BC, kFormNoConv>
                                                : (WaveSeqKernel)k_level_wave_seq<T, BC, kFormGeneral>);
  return (const void*)(form == kFormConstVisc ? (WaveKernel)k_level_wave<T, BC, kFormConstVisc>
                       : form == kFormNoConv  ? (WaveKernel)k_level_wave<T, BC, kFormNoConv>
                                              : (WaveKernel)k_level_wave<T, BC, kFormGeneral>);
}
const void* wave_kernel(const pts_problem* p, bool fp32, bool seq) {
  const bool per = p->bc == PTS_PERIODIC;
  const int f = flux_form(p);
  return fp32 ? (per ? wave_kernel_bc<float, 1>(f, seq) : wave_kernel_bc<float, 0>(f, seq))
              : (per ? wave_kernel_bc<double, 1>(f, seq) : wave_kernel_bc<double, 0>(f, seq));
}

// The batched wavefront kernel (instances of one problem in each launch).
typedef void (*WaveBatchKernel)(KProb, const WaveArgs*, Geo, int, int, int);
template <typename T, int BC>
WaveBatchKernel wave_batch_kernel_bc(int form) {
  return form == kFormConstVisc ? k_level_wave_batch<T, BC, kFormConstVisc>
         : form == kFormNoConv  ? k_level_wave_batch<T, BC, kFormNoConv>
                                : k_level_wave_batch<T, BC, kFormGeneral>;
}
WaveBatchKernel wave_batch_kernel(const pts_problem* p, bool fp32) {
  const bool per = p->bc == PTS_PERIODIC;
  const int f = flux_form(p);
  return fp32 ? (per ? wave_batch_kernel_bc<float, 1>(f) : wave_batch_kernel_bc<float, 0>(f))
              : (per ? wave_batch_kernel_bc<double, 1>(f) : wave_batch_kernel_bc<double, 0>(f));
}

// algorithmic bytes of anti-diagonal d: per active (stage, level) pair, U_j^n and
// U_{j+1}^{n-1} read, U_{j+1}^n written
double wave_bytes(const pts_problem* p, int stages, int d) {
  const int active = std::min(stages, d / 2 + 1) - std::max(0, (d - p->nt + 2) / 2);
  return 8.0 * 3.0 * (double)p->nx * p->ny * std::max(active, 0);
}

// Whether the cooperative form of a sequence fits: the device supports cooperative launches
// and holds every work-group at once (checked once per kernel and device).
bool wave_seq_fits(const void* kern, int blocks) {
  struct E {
    int dev;
    const void* k;
    int capacity;
  };
  static thread_local std::vector<E> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  for (const E& e : cache)
    if (e.dev == dev && e.k == kern) return blocks <= e.capacity;
  int coop = 0, cus = 0, per = 0;
  int cap = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kThreads, 0) == hipSuccess)
    cap = per * cus;
  cache.push_back({dev, kern, cap});
  return blocks <= cap;
}

// One cooperative launch for the whole sequence (k_level_wave_seq). *used = false when it
// does not fit the device (nothing launched; the caller launches per anti-diagonal).
int launch_wave_coop(const pts_problem* p, const KProb& kp, const WaveArgs& wa, const Geo& g, const Plan& pl,
                     hipStream_t s, Prof* pr, int* launches, unsigned* bar, unsigned spins, bool* used) {
  auto kern = wave_kernel(p, pl.fp32, true);
  const int blocks = wa.stages * tiles(p, g);
  *used = wave_seq_fits((const void*)kern, blocks);
  if (!*used) return PTS_OK;
  KProb a0 = kp;
  WaveArgs a1 = wa;
  Geo a2 = g;
  int ndiag = p->nt + 2 * (wa.stages - 1), passes = pl.passes, sweeps = pl.sweeps;
  void* args[] = {&a0, &a1, &a2, &ndiag, &passes, &sweeps, &bar, &spins};
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, (unsigned long long*)bar, 1);
  prof_begin(pr, 1, s);
  HIPCHK(hipLaunchCooperativeKernel((const void*)kern, dim3(blocks), dim3(kThreads), args, 0, s));
  if (pr) {
    for (int d = 0; d < ndiag; ++d) pr->bytes += wave_bytes(p, wa.stages, d);
    pr->end(s);
    pr->recs.back().count = ndiag;
  }
  *launches += 2;
  return PTS_OK;
}

int launch_wave_sequence(const pts_problem* p, const KProb& kp, const WaveArgs& wa, const Geo& g, const Plan& pl,
                         hipStream_t s, Prof* pr, int* launches) {
  const int tl = tiles(p, g);
  const int ndiag = p->nt + 2 * (wa.stages - 1);
  // profiling brackets the whole back-to-back sequence (per-launch events would add their
  // own overhead to every launch); the average launch is the interval over ndiag
  prof_begin(pr, 1, s);
  const WaveKernel kern = (WaveKernel)wave_kernel(p, pl.fp32, false);
  for (int d = 0; d < ndiag; ++d) {
    hipLaunchKernelGGL(kern, dim3(wa.stages * tl), dim3(kThreads), 0, s, kp, wa, g, d, pl.passes, pl.sweeps);
    if (pr) pr->bytes += wave_bytes(p, wa.stages, d);
    ++*launches;
  }
  if (pr) {
    pr->end(s);
    pr->recs.back().count = ndiag;
  }
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

// Replays the cached graph whose key matches, else captures `launch(stream)` into a new
// graph (on a capture stream of this thread) and replays that.
template <typename F>
int replay_or_capture(const std::vector<char>& key, hipStream_t s, int* launches, F&& launch) {
  for (auto& wg : g_wave_graphs) {
    if (wg.key == key) {
      HIPCHK(hipGraphLaunch(wg.exec, s));
      ++*launches;
      return PTS_OK;
    }
  }
  static thread_local hipStream_t cap = nullptr;
  if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = launch(cap);
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (rc) return rc;
  if (e != hipSuccess) return fail(PTS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  WaveGraph wg;
  e = hipGraphInstantiate(&wg.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(PTS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  wg.key = key;
  if (g_wave_graphs.size() >= 32) {  // drop the oldest
    (void)hipGraphExecDestroy(g_wave_graphs.front().exec);
    g_wave_graphs.erase(g_wave_graphs.begin());
  }
  g_wave_graphs.push_back(wg);
  HIPCHK(hipGraphLaunch(wg.exec, s));
  ++*launches;
  return PTS_OK;
}

// Appends the bytes of each value to a graph key.
template <typename... A>
void key_append(std::vector<char>& key, const A&... vals) {
  (key.insert(key.end(), (const char*)&vals, (const char*)&vals + sizeof(vals)), ...);
}

int run_wave_sequence(const pts_problem* p, const KProb& kp, const WaveArgs& wa, const Geo& g, const Plan& pl,
                      hipStream_t s, bool use_graph, Prof* pr, int* launches) {
  if (!use_graph || pr) return launch_wave_sequence(p, kp, wa, g, pl, s, pr, launches);
  // graphs are keyed on every launch argument; the solver passes u^0 through a workspace
  // copy, so for a given workspace they differ only with the caller's U
  std::vector<char> key;
  const int extra[4] = {0, pl.passes, pl.sweeps, pl.fp32 ? 1 : 0};  // extra[0]: one instance
  key_append(key, kp, wa, g, extra);
  return replay_or_capture(key, s, launches, [&](hipStream_t cs) -> int {
    int dummy = 0;
    return launch_wave_sequence(p, kp, wa, g, pl, cs, nullptr, &dummy);
  });
}

// Newton iterations overlapped in wavefront sequences of K stages each. Returns
// PTS_ERR_INVALID_ARG with *fallback = true when the inner solve does not fit the
// wavefront kernel (the caller then uses the bulk schedule).
int solve_wave(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
               const pts_options* o, pts_stats* st, hipStream_t s, bool* fallback, bool cplx) {
  *fallback = false;
  Instance in;
  in.bind(p, ws);
  Prof prof;
  const bool profiling = o && o->profile;
  if (profiling) in.prof = &prof;
  const bool use_graph = !profiling && (!o || o->use_graph != 0);
  double* hs;
  int rc = host_scalars(&hs);
  if (rc) return rc;
  char* wsb = (char*)ws;
  double* U1 = (double*)(wsb + in.L.U1);
  double* rho_part = (double*)(wsb + in.L.rho_part);
  double* res_part = (double*)(wsb + in.L.res_part);
  double* res_st = (double*)(wsb + in.L.res_st);
  double* u0w = (double*)(wsb + in.L.u0copy);
  HIPCHK(hipMemcpyAsync(u0w, u0, (size_t)p->nx * p->ny * 8, hipMemcpyDeviceToDevice, s));
  int launches = 0, it = 0;
  const size_t st_count = (size_t)p->nx * p->ny * p->nt;
  rc = in.residual(U, u0, s, &launches, false);
  if (rc) return rc;
  rc = in.read_scalars(hs, false, s);
  if (rc) return rc;
  double res = hs[0], rhom = hs[1];
  int needed = -1;  // Newton steps after which |R| <= tol was first seen
  Plan plan_used;
  for (;;) {
    if (st && it < PTS_MAX_HIST) {
      st->res_inf[it] = res;
      st->rho_max[it] = rhom;
    }
    if (!std::isfinite(res) || !std::isfinite(rhom)) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_NONFINITE, "non-finite residual at Newton step %d", it);
    }
    if (res <= tol && needed < 0) needed = it;
    if (res <= tol) break;
    if (level_solver(p, rhom, cplx) != 0) {
      if (it == 0) {  // the bulk schedule has the banded solve (or reports the error)
        *fallback = true;
        return PTS_ERR_INVALID_ARG;
      }
      if (st) st->iterations = it;
      return fail(PTS_ERR_NOT_DOMINANT, "Chebyshev level solves lost their convergence bound (Gershgorin radius "
                  "%.3g%s) at Newton step %d", rhom, cplx ? ", cell Peclet numbers above 2" : "", it);
    }
    if (it >= max_iter) {
      if (st) {
        st->iterations = it;
        st->launches = launches;
      }
      if (profiling) prof.collect(st);
      return fail(PTS_ERR_NOT_CONVERGED, "not converged after %d Newton steps (|R| = %.3e)", it, res);
    }
    Plan pl;
    int K = 1;
    if (!next_wave_plan(p, o, g_stage_cache.find(p, tol, ctag(o)), rhom, it, max_iter, &pl, &K)) {
      if (it == 0) {
        *fallback = true;
        return PTS_ERR_INVALID_ARG;
      }
      return fail(PTS_ERR_NOT_DOMINANT, "inner solve cannot reach the requested reduction (radius %.3g)", rhom);
    }
    const Geo g = in.g.whole ? in.g : geometry(p, wave_halo(pl));
    plan_used = pl;
    if (st) {
      st->sweeps = pl.sweeps;
      st->refine = pl.passes - 1;
      st->window = 1;
      st->schedule = PTS_SCHED_PIPELINE;
    }
    const int tl = tiles(p, g);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)(((K + 1) * tl + 255) / 256)), dim3(256), 0, s,
                       (unsigned long long*)res_part, (K + 1) * tl);
    launches += 1;
    WaveArgs wa;
    wa.Ur[0] = U;
    wa.Ur[1] = U1;
    wa.u0 = u0w;
    wa.rho_in = (const double*)in.rho;
    wa.rho_part = rho_part;
    wa.res_part = res_part;
    wa.tiles = tl;
    wa.stages = K;
    unsigned* bar = (unsigned*)(wsb + in.L.bar);
    bool coop = false;
    if (o && o->wave_launch == 1) {
      const unsigned spins = (o && o->barrier_spins > 0) ? (unsigned)o->barrier_spins : (1u << 20);
      rc = launch_wave_coop(p, in.kp, wa, g, pl, s, profiling ? &prof : nullptr, &launches, bar, spins, &coop);
      if (rc) return rc;
    }
    if (!coop) {
      rc = run_wave_sequence(p, in.kp, wa, g, pl, s, use_graph, profiling ? &prof : nullptr, &launches);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_stage_max, dim3(K + 1), dim3(256), 0, s, res_part, tl, res_st);
    ++launches;
    if (K & 1) {
      HIPCHK(hipMemcpyAsync(U, U1, st_count * 8, hipMemcpyDeviceToDevice, s));
    }
    // residuals of the iterates U_{it+1..it+K} formed by the stages; when the sequence
    // has not converged, the all-level residual of U_{it+K} also gives the radii with
    // which the next sequence starts
    HIPCHK(hipMemcpyAsync(hs + 8, res_st, (K + 1) * 8, hipMemcpyDeviceToHost, s));
    if (coop) HIPCHK(hipMemcpyAsync(hs + 40, bar, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (coop && ((const unsigned*)(hs + 40))[1] != 0) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_HIP, "wavefront sequence abandoned: a grid-barrier wait exceeded its poll limit");
    }
    for (int k = 1; k <= K; ++k) {
      const double rk = hs[8 + k];
      if (st && it + k < PTS_MAX_HIST) st->res_inf[it + k] = rk;
      if (rk <= tol && needed < 0) needed = it + k;
      if (!std::isfinite(rk)) {
        if (st) st->iterations = it + k;
        return fail(PTS_ERR_NONFINITE, "non-finite residual at Newton step %d", it + k);
      }
    }
    it += K;
    res = hs[8 + K];
    if (res > tol) {
      rc = in.residual(U, u0, s, &launches, false);
      if (rc) return rc;
      rc = in.read_scalars(hs, false, s);
      if (rc) return rc;
      res = hs[0];
      rhom = hs[1];
    }
    // the residual reported at `it` must be the one of the final iterate
    if (st && it < PTS_MAX_HIST) st->res_inf[it] = res;
    if (res <= tol) break;
  }
  if (needed >= 0 && plan_used.sweeps > 0) {
    // remember the step count for this plan (an autotuned plan stays the cached one)
    const StageCache::E* ce = g_stage_cache.find(p, tol, ctag(o));
    if (!ce || (ce->sweeps == plan_used.sweeps && ce->passes == plan_used.passes) || ce->sweeps == 0)
      g_stage_cache.put(p, tol, ctag(o), plan_used.sweeps, plan_used.passes, std::max(needed, 1), true);
  }
  if (st) {
    st->iterations = it;
    st->converged = 1;
    st->launches = launches;
  }
  if (profiling) prof.collect(st);
  return PTS_OK;
}


// Try inner plans for the wavefront schedule on this problem (each a full solve from the
// iterate in U, run twice: once to learn its Newton step count, once timed with HIP
// events on the stream) and cache the fastest. U is restored on return.
int autotune_wave(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
                  const pts_options* o, pts_stats* st, hipStream_t s) {
  bool cplx = false;
  {
    double* hs;
    int rc0 = host_scalars(&hs);
    if (!rc0) rc0 = convection_flag(p, u0, ws, s, hs, &cplx);
    if (rc0) return rc0;
  }
  Instance in;
  in.bind(p, ws);
  const size_t bytes = (size_t)p->nx * p->ny * p->nt * 8;
  double* backup = in.R;  // the residual array is not used by the wavefront schedule
  HIPCHK(hipMemcpyAsync(backup, U, bytes, hipMemcpyDeviceToDevice, s));
  const bool fp32 = p->precision == PTS_MIXED;
  std::vector<std::pair<int, int>> cands;
  if (!fp32) {
    for (int sw : {4, 5, 6, 7, 8, 10, 12, 16}) cands.push_back({sw, 1});
  } else {
    for (int sw : {3, 4, 5, 6}) cands.push_back({sw, 2});
    for (int sw : {3, 4}) cands.push_back({sw, 3});
    for (int sw : {5, 6, 8}) cands.push_back({sw, 1});
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best_sw = 0, best_pa = 0, best_steps = 0;
  pts_options oo = o ? *o : pts_options{};
  oo.schedule = PTS_SCHED_PIPELINE;
  oo.profile = 0;
  oo.lin_tol = 0;
  for (auto& c : cands) {
    oo.sweeps = c.first;
    oo.refine = c.second - 1;
    oo.stages = 0;
    Plan probe;
    probe.sweeps = c.first;
    probe.passes = c.second;
    if (!geometry(p).whole && wave_halo(probe) > kMaxWaveHalo) continue;
    // run 1: discover the step count (uncached plan -> stage guesses of 4)
    g_stage_cache.put(p, tol, ctag(o), c.first, c.second, 4);
    HIPCHK(hipMemcpyAsync(U, backup, bytes, hipMemcpyDeviceToDevice, s));
    bool fb = false;
    pts_stats s1;
    std::memset(&s1, 0, sizeof s1);
    pts_options o1 = oo;
    o1.sweeps = 0;
    o1.refine = -1;  // take the plan from the cache entry just written
    int rc = solve_wave(p, U, u0, tol, max_iter, ws, &o1, &s1, s, &fb, cplx);
    if (rc || !s1.converged) continue;
    const StageCache::E* ce = g_stage_cache.find(p, tol, ctag(o));
    const int steps = ce ? ce->steps : s1.iterations;
    // run 2: timed with the learned step count
    HIPCHK(hipMemcpyAsync(U, backup, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipEventRecord(e0, s));
    rc = solve_wave(p, U, u0, tol, max_iter, ws, &o1, &s1, s, &fb, cplx);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    if (rc || !s1.converged) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best_sw = c.first;
      best_pa = c.second;
      best_steps = steps;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipMemcpyAsync(U, backup, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (best_sw == 0) {
    g_stage_cache.put(p, tol, ctag(o), 0, 0, 0);
    return fail(PTS_ERR_NOT_CONVERGED, "autotune: no wavefront plan converged");
  }
  g_stage_cache.put(p, tol, ctag(o), best_sw, best_pa, best_steps);
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->sweeps = best_sw;
    st->refine = best_pa - 1;
    st->iterations = best_steps;
    st->solve_ms = best_ms;
    st->schedule = PTS_SCHED_PIPELINE;
    st->slab = p->nt;
  }
  return PTS_OK;
}


// One all-at-once Newton solve of `p` with the requested schedule (wavefront by default,
// bulk when the inner plan does not fit the wavefront kernel).
int solve_core(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
               const pts_options* o, pts_stats* st, hipStream_t s) {
  // variable steps (Eq. (3) with tau_n) run the bulk schedule
  if (p->dt_levels && o && o->schedule == PTS_SCHED_PIPELINE)
    return fail(PTS_ERR_INVALID_ARG, "the wavefront schedule takes uniform steps (dt_levels is set)");
  const int sched = ((o && o->window > 1) || p->dt_levels) ? PTS_SCHED_BULK : (o ? o->schedule : PTS_SCHED_AUTO);
  bool fallback = true, cplx = false;
  double* hs;
  int rc = host_scalars(&hs);
  if (!rc) rc = convection_flag(p, u0, ws, s, hs, &cplx);
  if (rc) return rc;
  if (sched != PTS_SCHED_BULK) {
    rc = solve_wave(p, U, u0, tol, max_iter, ws, o, st, s, &fallback, cplx);
    if (fallback && sched == PTS_SCHED_PIPELINE)
      rc = fail(PTS_ERR_INVALID_ARG, "the inner solve does not fit the wavefront schedule");
  }
  if (fallback && sched != PTS_SCHED_PIPELINE) {
    if (st) std::memset(st, 0, sizeof *st);
    rc = solve_bulk(p, U, u0, tol, max_iter, ws, o, st, s, false, cplx);
  }
  return rc;
}

// Divergence of plain Newton: a non-finite or exploding residual, or a block that lost
// diagonal dominance on the way.
bool diverged(int rc, const pts_stats& st) {
  if (rc == PTS_ERR_NONFINITE || rc == PTS_ERR_SINGULAR || rc == PTS_ERR_NOT_DOMINANT) return true;
  if (rc != PTS_ERR_NOT_CONVERGED) return false;
  const int n = std::min(st.iterations, PTS_MAX_HIST - 1);
  double mx = 0.0;
  for (int k = 0; k <= n; ++k) mx = std::max(mx, st.res_inf[k]);
  return !(mx <= 100.0 * st.res_inf[0]);
}

// Newton slab length that worked last time per problem signature (levels solved
// all-at-once together; nt = the whole space-time domain).
struct SlabCache {
  struct E {
    int nx, ny, nt, kind, bc, prec;
    double dt, mu_a, mu_b;
    int slab;
  };
  std::vector<E> v;
  int get(const pts_problem* p) const {
    for (auto& e : v)
      if (e.nx == p->nx && e.ny == p->ny && e.nt == p->nt && e.kind == p->kind && e.bc == p->bc &&
          e.prec == p->precision && e.dt == p->dt && e.mu_a == p->mu_a && e.mu_b == p->mu_b)
        return e.slab;
    return p->nt;
  }
  void put(const pts_problem* p, int slab) {
    for (auto& e : v)
      if (e.nx == p->nx && e.ny == p->ny && e.nt == p->nt && e.kind == p->kind && e.bc == p->bc &&
          e.prec == p->precision && e.dt == p->dt && e.mu_a == p->mu_a && e.mu_b == p->mu_b) {
        e.slab = slab;
        return;
      }
    if (v.size() > 64) v.clear();
    v.push_back({p->nx, p->ny, p->nt, p->kind, p->bc, p->precision, p->dt, p->mu_a, p->mu_b, slab});
  }
};
thread_local SlabCache g_slab_cache;

// All-at-once Newton over the whole space-time domain; if it diverges from the given
// iterate, the levels are solved in consecutive slabs, each all-at-once from the plain
// iterate of its own initial level, halving the slab until every slab converges (the
// root is the same: each slab's first level takes the previous slab's converged last
// level as u^{n-1}).
int solve_slabs(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
                const pts_options* o, pts_stats* st, hipStream_t s) {
  pts_stats local;
  pts_stats* sp = st ? st : &local;
  std::memset(sp, 0, sizeof *sp);
  int L = g_slab_cache.get(p);
  bool reinit = false;
  if (L >= p->nt) {
    int rc = solve_core(p, U, u0, tol, max_iter, ws, o, sp, s);
    sp->slab = p->nt;
    sp->hist = std::min(sp->iterations + 1, PTS_MAX_HIST);
    if (!diverged(rc, *sp)) return rc;
    L = std::max(1, p->nt / 2);
    reinit = true;
  }
  const size_t ns = (size_t)p->nx * p->ny;
  const int bstride = 2 * (p->nx + p->ny);
  int total_iters = 0, rc = PTS_OK;
  for (int s0 = 0; s0 < p->nt;) {
    pts_problem sub = *p;
    sub.nt = std::min(L, p->nt - s0);
    if (p->bdata) sub.bdata = p->bdata + (size_t)s0 * bstride;
    double* Us = U + (size_t)s0 * ns;
    const double* u0s = s0 == 0 ? u0 : U + (size_t)(s0 - 1) * ns;
    if (reinit) {
      const size_t total = ns * sub.nt;
      const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
      hipLaunchKernelGGL(k_broadcast, dim3(blocks), dim3(256), 0, s, ns, sub.nt, Us, u0s);
      HIPCHK(hipGetLastError());
    }
    std::memset(sp, 0, sizeof *sp);
    rc = solve_core(&sub, Us, u0s, tol, max_iter, ws, o, sp, s);
    if (diverged(rc, *sp)) {
      if (L == 1) return rc;
      L = std::max(1, L / 2);
      reinit = true;
      continue;  // redo this slab, shorter, from the plain iterate
    }
    total_iters += sp->iterations;
    sp->hist = std::min(sp->iterations + 1, PTS_MAX_HIST);
    if (rc) return rc;
    s0 += sub.nt;
  }
  g_slab_cache.put(p, L);
  sp->iterations = total_iters;
  sp->slab = L;
  return rc;
}

}  // namespace

// ------------------------------------------- Theorem 1 with explicit products (Section 5)
// Workspace of the explicit-product form (pts_newton_step_products): residual, rows of every
// A_n, two diamonds (P^{l-1}, P^l), the right-hand sides rt^l, the update, every level's band,
// reduction slots, the zero-pivot flag and the band descriptors.
struct ProdLayout {
  size_t R, coef, D0, D1, RT, RS, dU, lvl, scal, partial, rms, flag, desc, band, total;
  std::vector<size_t> B;  // band of level l
  std::vector<int> w;     // half-bandwidth of level l
};
int prod_w(const pts_problem* p, int l) {
  const long long ns = (long long)p->nx * p->ny;
  return (int)std::min<long long>((long long)l * p->nx, ns - 1);
}
ProdLayout prod_layout(const pts_problem* p) {
  ProdLayout L;
  const size_t ns = (size_t)p->nx * p->ny, st = ns * p->nt;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.R = take(st * 8);
  L.coef = take(st * 5 * 8);
  L.D0 = take((size_t)dia_count(p->nt) * ns * 8);
  L.D1 = take((size_t)dia_count(p->nt) * ns * 8);
  L.RT = take(st * 8);
  L.RS = take(st * 8);
  L.dU = take(st * 8);
  L.lvl = take((size_t)p->nt * 16);
  L.scal = take(4 * 8);
  L.partial = take(kUpdateBlocks * 8);
  L.rms = take(8);
  L.flag = take(8);
  L.desc = take((size_t)p->nt * sizeof(BandLevel));
  L.band = o;
  for (int l = 1; l <= p->nt; ++l) {
    L.w.push_back(prod_w(p, l));
    L.B.push_back(take(ns * (2 * (size_t)prod_w(p, l) + 1) * 8));
  }
  L.total = o;
  return L;
}
int prod_check(const pts_problem* p) {
  int rc = validate(p);
  if (rc) return rc;
  if (p->bc != PTS_DIRICHLET)
    return fail(PTS_ERR_INVALID_ARG, "explicit products: Dirichlet problems only (the band of a periodic grid wraps)");
  return PTS_OK;
}

// Residual and rows of every A_n at U (launch_residual), then the recursion of Section 5 up to
// level `upto`: rt^l and P^l (diamonds alternating between D0 and D1), and with `band` each
// P^l scaled by its diagonal into level l's band (the bands zeroed beforehand). *last points
// at the diamond of P^upto.
int prod_products(const pts_problem* p, const ProdLayout& L, char* ws, const double* U, const double* u0, int upto,
                  bool band, hipStream_t s, const double** last) {
  const size_t ns = (size_t)p->nx * p->ny;
  const KProb kp = kprob(p);
  double* R = (double*)(ws + L.R);
  double* coef = (double*)(ws + L.coef);
  double* RT = (double*)(ws + L.RT);
  int rc = launch_residual(p, kp, U, u0, R, coef, (unsigned long long*)(ws + L.lvl),
                           (unsigned long long*)(ws + L.scal), s);
  if (rc) return rc;
  double* D[2] = {(double*)(ws + L.D0), (double*)(ws + L.D1)};
  const unsigned nb = (unsigned)((ns + 255) / 256);
  for (int l = 1; l <= upto; ++l) {
    const double* Dp = D[(l + 1) & 1];
    double* Dc = D[l & 1];
    double* rt = RT + (size_t)(l - 1) * ns;
    hipLaunchKernelGGL(k_prod_rhs, dim3(nb), dim3(256), 0, s, p->nx, p->ny, l, Dp, R + (size_t)(l - 1) * ns,
                       l > 1 ? rt - ns : rt, rt);
    const size_t ne = (size_t)dia_count(l) * ns;
    hipLaunchKernelGGL(k_prod_level, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, p->nx, p->ny, l, Dp,
                       coef + (size_t)(l - 1) * 5 * ns, Dc);
    if (band)
      hipLaunchKernelGGL(k_prod_band, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, p->nx, p->ny, l,
                         L.w[l - 1], (const double*)Dc, (double*)(ws + L.B[l - 1]), (const double*)rt,
                         (double*)(ws + L.RS) + (size_t)(l - 1) * ns);
    *last = Dc;
  }
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

// One Newton step in the explicit-product form: assemble, scale and factor every level's
// P^l, solve, U += dU. res (host) receives max |R(U_in)|; the zero-pivot flag is checked.
int prod_step(const pts_problem* p, double* U, const double* u0, char* ws, const ProdLayout& L, pts_stats* st,
              int it, hipStream_t s, double* hs) {
  const size_t ns = (size_t)p->nx * p->ny;
  // band descriptors and zeroed bands, flag
  std::vector<BandLevel> bl(p->nt);
  for (int l = 1; l <= p->nt; ++l) bl[l - 1] = BandLevel{(double*)(ws + L.B[l - 1]), L.w[l - 1]};
  HIPCHK(hipMemcpyAsync(ws + L.desc, bl.data(), bl.size() * sizeof(BandLevel), hipMemcpyHostToDevice, s));
  {
    const size_t words = (L.total - L.band) / 8;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>((words + 255) / 256, 65535)), dim3(256), 0, s,
                       (unsigned long long*)(ws + L.band), (int)std::min<size_t>(words, 0x7fffffff));
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (unsigned long long*)(ws + L.flag), 1);
  }
  const double* last = nullptr;
  int rc = prod_products(p, L, ws, U, u0, p->nt, true, s, &last);
  if (rc) return rc;
  double* RS = (double*)(ws + L.RS);  // diagonally scaled right-hand sides
  // blocked band LU of every level, then the solves
  const BandLevel* dl = (const BandLevel*)(ws + L.desc);
  int* flag = (int*)(ws + L.flag);
  const int wmax = L.w.back();
  const int tmax = (wmax + 63) / 64;
  for (int k0 = 0; k0 < (int)ns; k0 += kPb) {
    hipLaunchKernelGGL(k_blu_panel, dim3((unsigned)p->nt), dim3(256), 0, s, dl, (int)ns, k0, flag);
    hipLaunchKernelGGL(k_blu_trsm, dim3((unsigned)((wmax + 255) / 256), (unsigned)p->nt), dim3(256), 0, s, dl,
                       (int)ns, k0);
    hipLaunchKernelGGL(k_blu_gemm, dim3((unsigned)(tmax * tmax), (unsigned)p->nt), dim3(256), 0, s, dl, (int)ns,
                       k0);
  }
  double* dU = (double*)(ws + L.dU);
  hipLaunchKernelGGL(k_blu_solve, dim3((unsigned)p->nt), dim3(256), 0, s, dl, (int)ns, (const double*)RS, dU);
  const size_t count = ns * p->nt;
  hipLaunchKernelGGL(k_update, dim3(kUpdateBlocks), dim3(256), 0, s, count, U, dU, (double*)(ws + L.partial));
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, (const double*)(ws + L.partial), kUpdateBlocks,
                     (double*)(ws + L.rms));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hs, ws + L.scal, 16, hipMemcpyDeviceToHost, s));  // max |R(U_in)|
  HIPCHK(hipMemcpyAsync(hs + 2, ws + L.rms, 8, hipMemcpyDeviceToHost, s));
  int fl = 0;
  HIPCHK(hipMemcpyAsync(&fl, flag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st && it < PTS_MAX_HIST) {
    st->res_inf[it] = hs[0];
    if (it + 1 < PTS_MAX_HIST) st->upd_rms[it + 1] = std::sqrt(hs[2] / (double)count);
  }
  if (!std::isfinite(hs[0])) return fail(PTS_ERR_NONFINITE, "explicit products: non-finite residual at step %d", it);
  if (fl) return fail(PTS_ERR_SINGULAR, "explicit products: zero pivot in the banded LU of a product P^l");
  return PTS_OK;
}

// ---------------------------------------------------------------- batched bulk solve
// Workspace of a batch: a header with the instance descriptors and the (instance, tile)
// work items, then every instance's own workspace.
// Dirichlet heat on square grids with equal spacings: the multigrid-preconditioned level
// solve applies.
bool mg_eligible(const pts_problem* probs, int nprob) {
  for (int i = 0; i < nprob; ++i) {
    const pts_problem& q = probs[i];
    if (q.kind != PTS_HEAT || q.bc != PTS_DIRICHLET || q.nx != q.ny || q.hx != q.hy || !(q.mu_a > 0) || q.dt_levels)
      return false;
  }
  return true;
}

// V-cycle hierarchy of an N x N grid for M = I + c (-Delta_h) (array pointers left NULL).
MgDesc mg_hierarchy(int N, double c) {
  MgDesc d;
  std::memset(&d, 0, sizeof d);
  int n = N, l = 0;
  d.G = -1;
  for (;;) {
    d.n[l] = n;
    d.a[l] = (float)(c * (double)(n + 1) * (double)(n + 1));
    if (d.G < 0 && n <= kMgLds) d.G = l;
    ++l;
    if (n <= kMgCoarsest || l == kMgLevels) break;
    n = mg_coarse(n);
  }
  d.levels = l;
  return d;
}

// Transfer tables of a hierarchy, grid after grid: k, w, own (n_l words each), sup (n_{l+1}
// int2), each array 16-byte aligned.
size_t mg_table_words(int n) { return (size_t)(n + 3) / 4 * 4; }
size_t mg_table_bytes(const MgDesc& h) {
  size_t b = 0;
  for (int l = 0; l + 1 < h.levels; ++l) b += 4 * (3 * mg_table_words(h.n[l]) + 2 * mg_table_words(h.n[l + 1]));
  return b;
}
// Fills the tables into host memory `host` and points h's table pointers at `dev`, the device
// copy of the same bytes.
void mg_fill_tables(MgDesc& h, char* host, char* dev) {
  size_t o = 0;
  for (int l = 0; l + 1 < h.levels; ++l) {
    const int nf = h.n[l], nc = h.n[l + 1];
    int* k = (int*)(host + o);
    float* w = (float*)(host + o + 4 * mg_table_words(nf));
    int* own = (int*)(host + o + 8 * mg_table_words(nf));
    int2* sup = (int2*)(host + o + 12 * mg_table_words(nf));
    mg_tables(nf, nc, k, w, own, sup);
    h.tk[l] = (const int*)(dev + o);
    h.tw[l] = (const float*)(dev + o + 4 * mg_table_words(nf));
    h.to[l] = (const int*)(dev + o + 8 * mg_table_words(nf));
    h.ts[l] = (const int2*)(dev + o + 12 * mg_table_words(nf));
    o += 4 * (3 * mg_table_words(nf) + 2 * mg_table_words(nc));
  }
}

// Tiles of grid l of a hierarchy for the down kernel (coarse tiles of grid l+1) and the up
// kernel (fine tiles of grid l).
int mg_down_tiles(const MgDesc& d, int l) {
  const int t = (d.n[l + 1] + kMgTC - 1) / kMgTC;
  return t * t;
}
int mg_up_tiles(const MgDesc& d, int l) {
  const int t = (d.n[l] + kMgTF - 1) / kMgTF;
  return t * t;
}

// Layout of the multigrid solve's part of a batch header (after the level-solve part).
// Every instance has kLanes level solvers ("lanes", descriptor index i kLanes + s): the bulk
// schedule uses lane 0; the pipelined schedule lanes 0..S-1 for its Newton stages and lane S
// for the update and residual after the last one (S <= kLanes - 1).
constexpr int kLanes = 8;
struct MgLayout {
  size_t desc, mgdesc, items_e, items_d, items_u, items_l, items_a, items_k, stat, total;
  size_t stat_words = 0;                        // [nt][3] per lane, lanes one after another
  std::vector<size_t> tab, lmax, lstat;         // per instance (lstat: its lane 0's stat words)
  std::vector<size_t> d, K, coef, R, ring, park;  // per lane
  std::vector<std::vector<size_t>> x, f, e;     // per lane, grids 0..G (e: 1..G-1)
  size_t ne = 0, nd = 0, nu = 0;                // work item capacities (all lanes)
  int gmax = 0;                                 // most grids above the LDS part
};
MgLayout mg_layout(const pts_problem* probs, int nprob) {
  MgLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  for (int i = 0; i < nprob; ++i) {
    const size_t N = probs[i].nx;
    L.ne += kLanes * std::max<size_t>(pc_tiles((int)N, (int)N), (N * N + 255) / 256);
    const MgDesc h = mg_hierarchy(probs[i].nx, probs[i].dt * probs[i].mu_a);
    for (int l = 0; l < h.G; ++l) {
      L.nd += kLanes * mg_down_tiles(h, l);
      L.nu += kLanes * mg_up_tiles(h, l);
    }
    L.gmax = std::max(L.gmax, h.G);
    L.lstat.push_back(L.stat_words);
    L.stat_words += (size_t)kLanes * kStat * probs[i].nt;
  }
  const size_t nl = (size_t)nprob * kLanes;
  L.desc = take(nl * sizeof(PcDesc));
  L.mgdesc = take(nl * sizeof(MgDesc));
  L.items_e = take(L.ne * sizeof(int2));
  L.items_a = take(L.ne * sizeof(int2));
  L.items_d = take(std::max<size_t>(L.nd, 1) * sizeof(int4));
  L.items_u = take(std::max<size_t>(L.nu, 1) * sizeof(int4));
  L.items_l = take(nl * sizeof(int));
  L.items_k = take(nl * sizeof(int));
  L.stat = take(L.stat_words * 8);
  L.x.resize(nl);
  L.f.resize(nl);
  L.e.resize(nl);
  for (int i = 0; i < nprob; ++i) {
    const size_t N = probs[i].nx, nt = probs[i].nt;
    const MgDesc h = mg_hierarchy(probs[i].nx, probs[i].dt * probs[i].mu_a);
    L.tab.push_back(take(mg_table_bytes(h)));
    L.lmax.push_back(take(nt * 8));
    for (int s = 0; s < kLanes; ++s) {
      const size_t q = (size_t)i * kLanes + s;
      for (int l = 0; l <= h.G; ++l) {
        const size_t nn = (size_t)h.n[l] * h.n[l];
        L.x[q].push_back(take(nn * 4));
        L.f[q].push_back(take(nn * 4));
        L.e[q].push_back(l >= 1 && l < h.G ? take(nn * 4) : 0);
      }
      L.d.push_back(take(N * N * 4));
      L.K.push_back(take(nt * 4));
      L.coef.push_back(take(nt * kMaxCheb * sizeof(float2)));
      L.R.push_back(take(N * N * 8));
      L.ring.push_back(take(2 * N * N * 4));
      L.park.push_back(take(N * N * 8));
    }
  }
  L.total = o;
  return L;
}

size_t batch_header_bytes(const pts_problem* probs, int nprob) {
  size_t tiles_total = 0;
  for (int i = 0; i < nprob; ++i) tiles_total += (size_t)tiles(probs + i, geometry(probs + i));
  size_t b = align_up((size_t)nprob * sizeof(BatchDesc)) + align_up(tiles_total * sizeof(int2));
  if (mg_eligible(probs, nprob)) b += mg_layout(probs, nprob).total;
  return b;
}

// Pinned staging for the descriptor upload (the batched solve synchronises every Newton step
// before it writes the staging again).
struct HostStage {
  char* h = nullptr;
  size_t n = 0;
  ~HostStage() {
    if (h) (void)hipHostFree(h);
  }
};
thread_local HostStage g_stage;
int host_stage(size_t bytes, char** out) {
  if (g_stage.n < bytes) {
    if (g_stage.h) HIPCHK(hipHostFree(g_stage.h));
    g_stage.h = nullptr;
    g_stage.n = 0;
    HIPCHK(hipHostMalloc((void**)&g_stage.h, bytes, hipHostMallocDefault));
    g_stage.n = bytes;
  }
  *out = g_stage.h;
  return PTS_OK;
}

// Newton steps each instance of a pipelined multigrid batch needed the last time the same batch
// (instances' kinds, sizes, coefficients, precision; the caller's cache tag) was solved to the
// same tolerance: the next solve gives each instance that many stages.
struct PassCache {
  std::vector<std::pair<unsigned long long, std::vector<int>>> v;  // per instance: Newton steps
  static unsigned long long key(const pts_problem* probs, int nprob, double tol, int tag) {
    unsigned long long h = 1469598103934665603ull;  // FNV-1a over the fields that fix the work
    auto mix = [&](const void* p, size_t n) {
      for (size_t i = 0; i < n; ++i) h = (h ^ ((const unsigned char*)p)[i]) * 1099511628211ull;
    };
    mix(&nprob, sizeof nprob);
    mix(&tol, sizeof tol);
    mix(&tag, sizeof tag);  // the caller's tag: starts of another kind need other step counts
    for (int i = 0; i < nprob; ++i) {
      const pts_problem& q = probs[i];
      const int iv[6] = {q.kind, q.bc, q.nx, q.ny, q.nt, q.precision};
      const double dv[5] = {q.hx, q.hy, q.dt, q.mu_a, q.mu_b};
      mix(iv, sizeof iv);
      mix(dv, sizeof dv);
    }
    return h;
  }
  const std::vector<int>* get(unsigned long long k) const {
    for (auto& e : v)
      if (e.first == k) return &e.second;
    return nullptr;
  }
  void put(unsigned long long k, const std::vector<int>& steps) {
    for (auto& e : v)
      if (e.first == k) {
        e.second = steps;
        return;
      }
    if (v.size() > 64) v.clear();
    v.push_back({k, steps});
  }
};
thread_local PassCache g_pass_cache;

// Pinned host buffer for the iteration counts the pipelined lanes plan (read every diagonal).
thread_local HostStage g_stage_k;
int host_stage_k(size_t bytes, int** out) {
  if (g_stage_k.n < bytes) {
    if (g_stage_k.h) HIPCHK(hipHostFree(g_stage_k.h));
    g_stage_k.h = nullptr;
    g_stage_k.n = 0;
    HIPCHK(hipHostMalloc((void**)&g_stage_k.h, bytes, hipHostMallocDefault));
    g_stage_k.n = bytes;
  }
  *out = (int*)g_stage_k.h;
  return PTS_OK;
}

// Newton on every instance at once: per step, the all-level residuals, then for each level n
// and launch l of the inner plans one launch over the tiles of every instance that has them
// (k_level_solve_batched), then the updates. Instances leave the batch when they converge.
// Stiff Dirichlet heat batches (Gershgorin radius >= kMgRho) solve their levels with the
// multigrid-preconditioned Chebyshev iteration instead (k_pc_*, k_mg_*), also in shared
// launches.
constexpr double kMgRho = 0.97;
int solve_batched_bulk(const pts_problem* probs, int nprob, double* const* U, const double* const* u0, double tol,
                       int max_iter, char* header, char* wsb, const pts_options* o, pts_stats* stats,
                       hipStream_t s) {
  std::vector<Instance> in(nprob);
  std::vector<int> ntiles(nprob);
  char* w = wsb;
  int maxnt = 0;
  size_t tiles_total = 0;
  for (int i = 0; i < nprob; ++i) {
    in[i].bind(probs + i, w);
    w += in[i].L.total;
    ntiles[i] = tiles(probs + i, in[i].g);
    tiles_total += ntiles[i];
    maxnt = std::max(maxnt, probs[i].nt);
    if (stats) std::memset(stats + i, 0, sizeof(pts_stats));
  }
  const bool eligible = mg_eligible(probs, nprob);
  BatchDesc* d_desc = (BatchDesc*)header;
  int2* d_items = (int2*)(header + align_up((size_t)nprob * sizeof(BatchDesc)));
  char* mg_base = header + align_up((size_t)nprob * sizeof(BatchDesc)) + align_up(tiles_total * sizeof(int2));
  MgLayout DL;
  if (eligible) DL = mg_layout(probs, nprob);
  // host staging: descriptors and items of both solvers, then the scalars read back
  size_t so = 0;
  auto stake = [&](size_t bytes) {
    const size_t at = so;
    so = align_up(so + bytes);
    return at;
  };
  const size_t s_desc = stake((size_t)nprob * sizeof(BatchDesc)), s_items = stake(tiles_total * sizeof(int2));
  const size_t nlanes = (size_t)nprob * kLanes;
  const size_t s_dd = stake(eligible ? nlanes * sizeof(PcDesc) : 0);
  const size_t s_mg = stake(eligible ? nlanes * sizeof(MgDesc) : 0);
  const size_t s_id = stake(eligible ? DL.nd * sizeof(int4) : 0);
  const size_t s_iu = stake(eligible ? DL.nu * sizeof(int4) : 0);
  const size_t s_il = stake(eligible ? nlanes * sizeof(int) : 0);
  const size_t s_ie = stake(eligible ? DL.ne * sizeof(int2) : 0);
  const size_t s_ia = stake(eligible ? DL.ne * sizeof(int2) : 0);
  size_t tab_bytes = 0;
  if (eligible)
    for (int i = 0; i < nprob; ++i) tab_bytes += mg_table_bytes(mg_hierarchy(probs[i].nx, probs[i].dt * probs[i].mu_a));
  const size_t s_tab = stake(tab_bytes);
  size_t sum_nt = 0;
  for (int i = 0; i < nprob; ++i) sum_nt += probs[i].nt;
  const size_t s_kt = stake(eligible ? sum_nt * 4 : 0);
  const size_t s_cf = stake(eligible ? sum_nt * kMaxCheb * sizeof(float2) : 0);
  const size_t s_lm = stake(eligible ? sum_nt * 8 : 0);
  const size_t s_sc = stake((size_t)nprob * 4 * sizeof(double));
  char* stage;
  int rc = host_stage(so, &stage);
  if (rc) return rc;
  BatchDesc* h_desc = (BatchDesc*)(stage + s_desc);
  int2* h_items = (int2*)(stage + s_items);
  PcDesc* h_dd = (PcDesc*)(stage + s_dd);
  MgDesc* h_mg = (MgDesc*)(stage + s_mg);
  int4* h_id = (int4*)(stage + s_id);
  int4* h_iu = (int4*)(stage + s_iu);
  int* h_il = (int*)(stage + s_il);
  int2* h_ie = (int2*)(stage + s_ie);
  int2* h_ia = (int2*)(stage + s_ia);
  double* h_sc = (double*)(stage + s_sc);  // per instance: max|r|, rho_max, rms, max|u^0|
  std::vector<size_t> ofs_nt(nprob, 0);      // instance i's levels start at ofs_nt[i] in the per-level tables
  for (int i = 1; i < nprob; ++i) ofs_nt[i] = ofs_nt[i - 1] + probs[i - 1].nt;
  int* h_kt = (int*)(stage + s_kt);
  float2* h_cf = (float2*)(stage + s_cf);
  double* h_lm = (double*)(stage + s_lm);
  bool use_mg = false;
  // profiling (pts_options.profile): every launch of the multigrid-preconditioned level solves
  // bracketed by HIP events, the intervals collected after each Newton step
  Prof prof_obj;
  Prof* prof = (o && o->profile) ? &prof_obj : nullptr;
  pts_stats pstat;
  std::memset(&pstat, 0, sizeof pstat);
  const bool fp32 = probs[0].precision == PTS_MIXED;
  const bool per = probs[0].bc == PTS_PERIODIC;
  auto kern = fp32 ? (per ? k_level_solve_batched<float, 1> : k_level_solve_batched<float, 0>)
                   : (per ? k_level_solve_batched<double, 1> : k_level_solve_batched<double, 0>);

  std::vector<char> active(nprob, 1);
  std::vector<Plan> plans(nprob);
  int launches = 0, worst = PTS_OK;
  auto read_all = [&](bool with_rms, bool with_u0, bool with_levels) -> int {
    for (int i = 0; i < nprob; ++i) {
      if (!active[i]) continue;
      HIPCHK(hipMemcpyAsync(h_sc + 4 * i, in[i].scal, 16, hipMemcpyDeviceToHost, s));
      if (with_rms) HIPCHK(hipMemcpyAsync(h_sc + 4 * i + 2, in[i].rms, 8, hipMemcpyDeviceToHost, s));
      if (with_u0) HIPCHK(hipMemcpyAsync(h_sc + 4 * i + 3, in[i].scal + 3, 8, hipMemcpyDeviceToHost, s));
      if (with_levels)
        HIPCHK(hipMemcpyAsync(h_lm + ofs_nt[i], mg_base + DL.lmax[i], (size_t)probs[i].nt * 8, hipMemcpyDeviceToHost,
                              s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return PTS_OK;
  };
  // max |u^n| per level of the current iterate (the spectral solve's Chebyshev intervals)
  auto level_max = [&](int i) {
    hipLaunchKernelGGL(k_level_absmax, dim3((unsigned)probs[i].nt), dim3(256), 0, s, U[i],
                       (size_t)probs[i].nx * probs[i].ny, (unsigned long long*)(mg_base + DL.lmax[i]));
    ++launches;
  };
  // the initial residual's maxima (convergence, Gershgorin radius, level maxima); the pipelined
  // multigrid lanes form each level's residual themselves, so a batch that may take them stores
  // none here (and forms it again below if its blocks turn out not to be stiff)
  const bool may_pipe = eligible && (o == nullptr || o->schedule != PTS_SCHED_BULK);
  for (int i = 0; i < nprob; ++i) {
    if ((rc = in[i].residual(U[i], u0[i], s, &launches, !may_pipe))) return rc;
    if (eligible) level_max(i);
  }
  if ((rc = read_all(false, false, eligible))) return rc;
  double rho0 = 0.0;
  for (int i = 0; i < nprob; ++i) rho0 = std::max(rho0, h_sc[4 * i + 1]);
  use_mg = eligible && rho0 >= kMgRho;
  if (may_pipe && !use_mg)
    for (int i = 0; i < nprob; ++i)
      if ((rc = in[i].residual(U[i], u0[i], s, &launches))) return rc;
  if (use_mg) {
    // hierarchies (fixed for the solve): one transfer table per instance, grids per lane
    size_t to = 0;
    for (int i = 0; i < nprob; ++i) {
      MgDesc m = mg_hierarchy(probs[i].nx, probs[i].dt * probs[i].mu_a);
      const size_t tb = mg_table_bytes(m);
      mg_fill_tables(m, stage + s_tab + to, mg_base + DL.tab[i]);
      HIPCHK(hipMemcpyAsync(mg_base + DL.tab[i], stage + s_tab + to, tb, hipMemcpyHostToDevice, s));
      to += tb;
      for (int ln = 0; ln < kLanes; ++ln) {
        const size_t q = (size_t)i * kLanes + ln;
        for (int l = 0; l <= m.G; ++l) {
          m.x[l] = (float*)(mg_base + DL.x[q][l]);
          m.f[l] = (float*)(mg_base + DL.f[q][l]);
          m.e[l] = l >= 1 && l < m.G ? (float*)(mg_base + DL.e[q][l]) : nullptr;
        }
        h_mg[q] = m;
      }
    }
    HIPCHK(hipMemcpyAsync(mg_base + DL.mgdesc, h_mg, nlanes * sizeof(MgDesc), hipMemcpyHostToDevice, s));
  }
  // descriptor of lane ln of instance i (pipelined lanes set their stage fields afterwards)
  auto lane_desc = [&](int i, int ln) {
    PcDesc d;
    std::memset(&d, 0, sizeof d);
    const size_t q = (size_t)i * kLanes + ln;
    d.p = in[i].kp;
    d.U = U[i];
    d.R = in[i].R;
    d.dU = in[i].dU;
    d.r = (float*)(mg_base + DL.f[q][0]);
    d.z = (float*)(mg_base + DL.x[q][0]);
    d.d = (float*)(mg_base + DL.d[q]);
    d.K = (int*)(mg_base + DL.K[q]);
    d.c = (float2*)(mg_base + DL.coef[q]);
    d.active = active[i];
    d.ld = probs[i].nx;
    d.rmask = -1;
    d.dmask = -1;
    d.u0 = u0[i];
    d.stat = (unsigned long long*)(mg_base + DL.stat) + DL.lstat[i] + (size_t)ln * kStat * probs[i].nt;
    return d;
  };
  const double lin_tol = (o && o->lin_tol > 0) ? o->lin_tol : 1e-3;
  const bool pipelined = o == nullptr || o->schedule != PTS_SCHED_BULK;
  const unsigned long long skey = PassCache::key(probs, nprob, tol, ctag(o));
  const std::vector<int>* cached = g_pass_cache.get(skey);
  // stages per pass of instance i: asked for; else from the Newton steps it needed last time,
  // split into as many passes as the instance that needed the most takes (at most kLanes - 1
  // stages each); else kLanes - 1
  int cmax = 0;
  if (cached)
    for (int c : *cached) cmax = std::max(cmax, c);
  const int npass_c = cmax > 0 ? (cmax + kLanes - 2) / (kLanes - 1) : 1;
  std::vector<int> nstages(nprob, kLanes - 1);
  const bool from_cache = !(o && o->stages > 0) && cmax > 0;
  std::vector<int> cache_old = from_cache ? *cached : std::vector<int>();
  for (int i = 0; i < nprob; ++i) {
    if (o && o->stages > 0)
      nstages[i] = std::min(kLanes - 1, o->stages);
    else if (from_cache)
      nstages[i] = std::min(kLanes - 1, std::max(1, (cache_old[i] + npass_c - 1) / npass_c));
  }
  std::vector<int> conv_it(nprob, -1);  // Newton step at which each instance met tol (pipelined)
  std::vector<int> done(nprob, 0);      // Newton steps applied to each instance
  bool was_pass = false;                // the last step was a pipelined pass (done[] advanced)
  for (int it = 0;; ++it) {
    if (it > 0 && !was_pass)
      for (int i = 0; i < nprob; ++i)
        if (active[i]) ++done[i];
    was_pass = false;
    int nactive = 0;
    for (int i = 0; i < nprob; ++i) {
      if (!active[i]) continue;
      const pts_problem* p = probs + i;
      const double res = h_sc[4 * i], rhom = h_sc[4 * i + 1];
      pts_stats* st = stats ? stats + i : nullptr;
      const int ki = done[i];
      if (st) {
        if (ki < PTS_MAX_HIST) {
          st->res_inf[ki] = res;
          st->rho_max[ki] = rhom;
          if (ki > 0) st->upd_rms[ki] = std::sqrt(h_sc[4 * i + 2] / ((double)p->nx * p->ny * p->nt));
        }
        st->iterations = ki;
        st->hist = std::min(ki + 1, PTS_MAX_HIST);
        st->slab = p->nt;
        st->window = 1;
        st->schedule = use_mg && pipelined ? PTS_SCHED_PIPELINE : PTS_SCHED_BULK;
      }
      int err = PTS_OK;
      if (!std::isfinite(res) || !std::isfinite(rhom)) {
        err = fail(PTS_ERR_NONFINITE, "instance %d: non-finite residual at Newton step %d", i, ki);
      } else if (res <= tol) {
        if (st) st->converged = 1;
        active[i] = 0;
        continue;
      } else if (rhom >= 1.0) {
        err = fail(PTS_ERR_NOT_DOMINANT, "instance %d: block not diagonally dominant (radius %.3g)", i, rhom);
      } else if (ki >= max_iter) {
        err = fail(PTS_ERR_NOT_CONVERGED, "instance %d: not converged after %d Newton steps (|R| = %.3e)", i, ki,
                   res);
      }
      if (err) {
        if (!worst) worst = err;
        active[i] = 0;
        continue;
      }
      if (!use_mg) {
        plans[i] = make_plan(p, o, std::min(rhom * 1.02, 0.999), in[i].g);
        if (st) {
          st->sweeps = plans[i].sweeps;
          st->refine = plans[i].passes - 1;
        }
      }
      ++nactive;
    }
    if (nactive == 0) break;
    std::vector<int> order;
    for (int i = 0; i < nprob; ++i)
      if (active[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].nt > probs[b].nt; });
    // per level n: the instances with nt > n form a prefix of `order`
    std::vector<int> kpref(maxnt, 0);
    for (int n = 0, k = (int)order.size(); n < maxnt; ++n) {  // the prefix shrinks as n grows
      while (k > 0 && probs[order[k - 1]].nt <= n) --k;
      kpref[n] = k;
    }
    // grids of the tile kernels: a multiple of the 8 XCDs, so that the kernels hand each XCD one
    // contiguous band of work items (xcd_band); the surplus work-groups return
    auto grid8 = [](size_t n) { return dim3((unsigned)((n + kXcds - 1) / kXcds * kXcds)); };
    // profiling brackets of the multigrid launches (kinds: pts_stats.kern_* slots)
    auto pb = [&](int kind) { prof_begin(prof, Prof::kKern + kind, s); };
    auto pe = [&](double bytes) {
      if (prof) {
        prof->end(s);
        prof->recs.back().bytes = bytes;
      }
    };
    const int gmax = use_mg ? DL.gmax : 0;
    const PcDesc* dd = (const PcDesc*)(mg_base + DL.desc);
    const MgDesc* dm = (const MgDesc*)(mg_base + DL.mgdesc);
    const int2* ie = (const int2*)(mg_base + DL.items_e);
    const int2* ia = (const int2*)(mg_base + DL.items_a);
    const int4* id = (const int4*)(mg_base + DL.items_d);
    const int4* iu = (const int4*)(mg_base + DL.items_u);
    const int* il = (const int*)(mg_base + DL.items_l);
    // algorithmic bytes per node of the grid a launch works on (profiling), for lane q (index
    // i kLanes + s) of instance i at Chebyshev iteration kk (x, du: xb bytes each): k_pc_resid
    // at kk = 0 reads r^n and du^{n-1}, writes b = r^n + du^{n-1} over r^n, x = 0 and r, at
    // kk > 0 reads b, u^n (8 each), x and writes r (4); k_mg_down reads f_l, writes x_l
    // and f_{l+1} (a quarter node); k_mg_lds reads f_G, writes x_G; k_mg_up reads x_l, f_l,
    // x_{l+1} and writes e_l, on the finest grid instead the Chebyshev step's reads and writes
    // of d (4 each) and du^n; where k_mg_lds holds the whole V-cycle (G = 0) it reads r and takes
    // that step (the pipelined lanes hold x and du in float32: xb = 4 bytes per node, else 8)
    auto kb = [&](int kind, int i, int kk, int g, double xb) {
      const MgDesc& m = h_mg[(size_t)i * kLanes];
      const double N2 = (double)probs[i].nx * probs[i].nx;
      const int l = g - (gmax - m.G);
      const double step = 8.0 + 2.0 * xb;  // the Chebyshev step, per node
      switch (kind) {
        case 0: return N2 * (kk == 0 ? 20.0 + 2.0 * xb : 20.0 + xb);
        case 1: return l >= 0 ? (double)m.n[l] * m.n[l] * 8.0 + (double)m.n[l + 1] * m.n[l + 1] * 4.0 : 0.0;
        case 2: return m.G == 0 ? N2 * (4.0 + step) : (double)m.n[m.G] * m.n[m.G] * 8.0;
        case 3:
          return l >= 0 ? (double)m.n[l] * m.n[l] * (l == 0 ? 8.0 + step : 12.0) +
                              (double)m.n[l + 1] * m.n[l + 1] * 4.0
                        : 0.0;
        default: return N2 * (kk == 0 ? 8.0 + 2.0 * xb : 12.0 + 2.0 * xb);
      }
    };
    // the V-cycle launches of Chebyshev iteration kk for the first ks lanes of a lane order
    // (k_pc_resid, the down kernels, the LDS part, the up kernels; the last of them applies the
    // Chebyshev step on the finest grid, k_mg_lds where the whole V-cycle is in LDS); m is the level
    // (bulk) or the diagonal (pipelined); bytes(kind, g) gives the profiled launches' bytes
    auto vcycle = [&](int m, int kk, bool resid, size_t ks, const std::vector<size_t>& ce,
                      const std::vector<std::vector<size_t>>& cd, const std::vector<std::vector<size_t>>& cu,
                      const std::vector<size_t>& od, const std::vector<size_t>& ou, auto&& bytes) {
      if (resid) {
        pb(0);
        hipLaunchKernelGGL(k_pc_resid, grid8(ce[ks]), dim3(256), 0, s, dd, ie, m, kk, (int)ce[ks]);
        pe(prof ? bytes(0, 0) : 0.0);
        ++launches;
      }
      for (int g = 0; g < gmax; ++g) {
        if (!cd[g][ks]) continue;
        pb(1);
        hipLaunchKernelGGL(k_mg_down, grid8(cd[g][ks]), dim3(kMgThreads), 0, s, dm, dd, id + od[g], m, kk,
                           (int)cd[g][ks]);
        pe(prof ? bytes(1, g) : 0.0);
        ++launches;
      }
      pb(2);
      hipLaunchKernelGGL(k_mg_lds, dim3((unsigned)ks), dim3(1024), 0, s, dm, dd, il, m, kk);
      pe(prof ? bytes(2, 0) : 0.0);
      ++launches;
      for (int g = gmax - 1; g >= 0; --g) {
        if (!cu[g][ks]) continue;
        pb(3);
        hipLaunchKernelGGL(k_mg_up, grid8(cu[g][ks]), dim3(kMgThreads), 0, s, dm, dd, iu + ou[g], m, kk,
                           (int)cu[g][ks]);
        pe(prof ? bytes(3, g) : 0.0);
        ++launches;
      }
    };
    // work items of a lane order: node tiles (ce), lane ids, and per step g the down/up tiles (an
    // instance takes part when g >= gmax - G_i, on grid g - (gmax - G_i)); cumulative counts
    // per prefix of the order, the items uploaded to the header
    auto build_items = [&](const std::vector<int>& lanes, std::vector<size_t>& ce,
                           std::vector<std::vector<size_t>>& cd, std::vector<std::vector<size_t>>& cu,
                           std::vector<size_t>& od, std::vector<size_t>& ou) -> int {
      const size_t no = lanes.size();
      ce.assign(no + 1, 0);
      cd.assign(gmax, std::vector<size_t>(no + 1, 0));
      cu = cd;
      od.assign(gmax, 0);
      ou.assign(gmax, 0);
      size_t ne = 0, nd = 0, nu = 0;
      for (size_t q = 0; q < no; ++q) {
        const int ln = lanes[q], i = ln / kLanes;
        const int N = probs[i].nx, ch = pc_tiles(N, N);
        for (int c = 0; c < ch; ++c) h_ie[ne++] = make_int2(ln, c);
        ce[q + 1] = ne;
        h_il[q] = ln;
      }
      for (int g = 0; g < gmax; ++g) {
        od[g] = nd;
        ou[g] = nu;
        for (size_t q = 0; q < no; ++q) {
          const int ln = lanes[q];
          const MgDesc& m = h_mg[ln];
          const int l = g - (gmax - m.G);
          if (l >= 0) {
            const int td = (m.n[l + 1] + kMgTC - 1) / kMgTC, tu = (m.n[l] + kMgTF - 1) / kMgTF;
            for (int ty = 0; ty < td; ++ty)
              for (int tx = 0; tx < td; ++tx) h_id[nd++] = make_int4(ln, l, tx, ty);
            for (int ty = 0; ty < tu; ++ty)
              for (int tx = 0; tx < tu; ++tx) h_iu[nu++] = make_int4(ln, l, tx, ty);
          }
          cd[g][q + 1] = nd - od[g];
          cu[g][q + 1] = nu - ou[g];
        }
      }
      HIPCHK(hipMemcpyAsync(mg_base + DL.desc, h_dd, nlanes * sizeof(PcDesc), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(mg_base + DL.items_e, h_ie, ne * sizeof(int2), hipMemcpyHostToDevice, s));
      if (nd) HIPCHK(hipMemcpyAsync(mg_base + DL.items_d, h_id, nd * sizeof(int4), hipMemcpyHostToDevice, s));
      if (nu) HIPCHK(hipMemcpyAsync(mg_base + DL.items_u, h_iu, nu * sizeof(int4), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(mg_base + DL.items_l, h_il, no * sizeof(int), hipMemcpyHostToDevice, s));
      return PTS_OK;
    };
    if (use_mg && pipelined) {
      // S_i Newton steps of instance i in one pass over the diagonals D = n + s (k_pipe_* kernels):
      // lanes (i, s), s = 0..S_i, ordered by nt_i + s, longest first; lane (i, s) has a level at
      // D while D < nt_i + s, so the lanes of a diagonal are a prefix of the order (lanes with
      // D < s return at once)
      std::vector<int> Si(nprob, 0);
      int S = 0;
      for (int i : order) {
        // a pass after the stages the cache predicted: the prediction fell short by little (the
        // residual of a step near tol varies with the start), two more stages
        const int want = from_cache && done[i] > 0 && done[i] >= cache_old[i] ? 2 : nstages[i];
        Si[i] = std::min(want, std::max(1, max_iter - done[i]));  // no more steps than max_iter allows
        S = std::max(S, Si[i]);
      }
      std::vector<int> all, solving;
      for (int i : order)
        for (int sg = 0; sg <= Si[i]; ++sg) all.push_back(i * kLanes + sg);
      auto key = [&](int ln) { return probs[ln / kLanes].nt + ln % kLanes; };
      std::stable_sort(all.begin(), all.end(), [&](int a, int b) { return key(a) > key(b); });
      for (int ln : all)
        if (ln % kLanes < Si[ln / kLanes]) solving.push_back(ln);
      // each lane plans its level's iterations from that level's max |u| (k_pipe_cheb); the
      // host reads the plans back and launches the most any lane needs. A lane's plan is
      // capped at the plan for twice the largest level maximum of the iterate the pass starts
      // from and the tightest reduction a lane asks, lin_tol / 10 (the heat iterates do not
      // grow: the cap only bounds a run-away iterate's work).
      int kcap = 1;
      for (int i : order) {
        double um = 0.0;
        for (int n = 0; n < probs[i].nt; ++n) um = std::max(um, h_lm[ofs_nt[i] + n]);
        float2 c[kMaxCheb];
        kcap = std::max(kcap, mg_cheb_plan(probs[i].mu_a, probs[i].mu_b, 2.0 * um, lin_tol / 10.0, c));
      }
      for (int i = 0; i < nprob; ++i)
        for (int ln = 0; ln < kLanes; ++ln) {
          const size_t q = (size_t)i * kLanes + ln;
          PcDesc d = lane_desc(i, ln);
          d.active = active[i] && ln <= Si[i];
          d.stage = ln;
          d.rmask = 0;
          d.dmask = 1;
          d.last = ln == Si[i];
          d.R = (double*)(mg_base + DL.R[q]);
          d.dU = nullptr;
          d.dxf = (float*)(mg_base + DL.ring[q]);
          d.park_out = ln >= 1 ? (double*)(mg_base + DL.park[q - 1]) : nullptr;
          d.park_in = ln < Si[i] ? (const double*)(mg_base + DL.park[q]) : nullptr;
          d.dprev = ln >= 1 ? (const float*)(mg_base + DL.ring[q - 1]) : nullptr;
          d.tgt = lin_tol;
          d.ntol = tol / 3.0;
          d.kcap = kcap;
          h_dd[q] = d;
        }
      std::vector<size_t> ce, od, ou;
      std::vector<std::vector<size_t>> cd, cu;
      if ((rc = build_items(solving, ce, cd, cu, od, ou))) return rc;
      // node tiles of every lane (the update and residual launches)
      std::vector<size_t> ca(all.size() + 1, 0);
      size_t na = 0;
      for (size_t q = 0; q < all.size(); ++q) {
        const int N = probs[all[q] / kLanes].nx, ch = pc_tiles(N, N);
        for (int c = 0; c < ch; ++c) h_ia[na++] = make_int2(all[q], c);
        ca[q + 1] = na;
      }
      HIPCHK(hipMemcpyAsync(mg_base + DL.items_a, h_ia, na * sizeof(int2), hipMemcpyHostToDevice, s));
      unsigned long long* stat = (unsigned long long*)(mg_base + DL.stat);
      hipLaunchKernelGGL(k_zero, dim3((unsigned)((DL.stat_words + 255) / 256)), dim3(256), 0, s, stat,
                         (int)DL.stat_words);
      ++launches;
      // the iteration counts the lanes planned, read back per diagonal
      int* kq = nullptr;
      if ((rc = host_stage_k(solving.size() * sizeof(int), &kq))) return rc;
      int kmax_all = 0;
      int* d_kq = (int*)(mg_base + DL.items_k);
      auto lane_level = [&](int ln, int D) {
        const int n = D - ln % kLanes;
        return (n >= 0 && n < probs[ln / kLanes].nt) ? n : -1;
      };
      const int Dend = key(all.front());
      size_t ka = all.size(), ks = solving.size();
      for (int D = 0; D < Dend; ++D) {
        while (ka > 0 && key(all[ka - 1]) <= D) --ka;
        while (ks > 0 && key(solving[ks - 1]) <= D) --ks;
        double b5 = 0.0, b6 = 0.0;
        if (prof)
          for (size_t q = 0; q < ka; ++q) {
            const int ln = all[q], sg = ln % kLanes;
            if (lane_level(ln, D) < 0) continue;
            const double N2 = (double)probs[ln / kLanes].nx * probs[ln / kLanes].nx;
            b5 += N2 * (sg == Si[ln / kLanes] ? 16.0 : 24.0);  // reads u^n, u^{n-1}; writes r
            if (sg >= 1) b6 += N2 * 28.0;        // reads u^n, du (float32); writes the park and u^n
          }
        pb(6);
        hipLaunchKernelGGL(k_pipe_update, grid8(ca[ka]), dim3(256), 0, s, dd, ia, D, (int)ca[ka]);
        pe(b6);
        pb(5);
        hipLaunchKernelGGL(k_pipe_residual, grid8(ca[ka]), dim3(256), 0, s, dd, ia, D, (int)ca[ka]);
        pe(b5);
        launches += 2;
        if (ks == 0) continue;
        // the first iteration's residual, from x0 = du^{n-1} (n > 0), before the plans
        double b0 = 0.0;
        if (prof)
          for (size_t q = 0; q < ks; ++q) {
            const int ln = solving[q], n = lane_level(ln, D);
            if (n < 0) continue;
            const double N2 = (double)probs[ln / kLanes].nx * probs[ln / kLanes].nx;
            b0 += N2 * (n > 0 ? 36.0 : 24.0);  // r^n (read and rewritten as b), u^n, du^{n-1}, x, r
          }
        pb(0);
        hipLaunchKernelGGL(k_pc_resid, grid8(ce[ks]), dim3(256), 0, s, dd, ie, D, 0, (int)ce[ks]);
        pe(b0);
        ++launches;
        pb(7);
        hipLaunchKernelGGL(k_pipe_cheb, dim3((unsigned)((ks + 63) / 64)), dim3(64), 0, s, dd, il, (int)ks, D, d_kq);
        pe(0.0);
        ++launches;
        HIPCHK(hipMemcpyAsync(kq, d_kq, ks * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int kn = 0;
        for (size_t q = 0; q < ks; ++q) kn = std::max(kn, kq[q]);
        kmax_all = std::max(kmax_all, kn);
        for (int kk = 0; kk < kn; ++kk)
          vcycle(D, kk, kk > 0, ks, ce, cd, cu, od, ou, [&](int kind, int g) {
            double b = 0.0;
            for (size_t q = 0; q < ks; ++q)
              if (lane_level(solving[q], D) >= 0 && kk < kq[q]) b += kb(kind, solving[q] / kLanes, kk, g, 4.0);
            return b;
          });
      }
      HIPCHK(hipGetLastError());
      // the result: max |R| of U^(S_i) (lane S_i), the largest radius and any NaN of every lane
      std::vector<unsigned long long> hst(DL.stat_words);
      HIPCHK(hipMemcpyAsync(hst.data(), stat, DL.stat_words * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      auto val = [](unsigned long long b) {
        double v;
        std::memcpy(&v, &b, 8);
        return v;
      };
      // stages the pass needed: per instance the first s whose iterate meets tol at every level
      bool all_met = true;
      for (int i : order) {
        const unsigned long long* st = hst.data() + DL.lstat[i];
        const int nt = probs[i].nt;
        int first = -1;
        for (int sg = 0; sg <= Si[i] && first < 0; ++sg) {
          unsigned long long r = 0;
          for (int n = 0; n < nt; ++n) r = std::max(r, st[((size_t)sg * nt + n) * kStat + 1]);
          if (val(r) <= tol) first = sg;
        }
        if (first < 0)
          all_met = false;
        else
          conv_it[i] = done[i] + first;
      }
      // all instances met tol: keep the Newton steps each instance needed (from its first
      // iterate), never fewer than kept before (a pass that falls short costs a sweep over
      // every diagonal of the instance; a stage too many costs one level solve per level)
      if (all_met && !(o && o->stages > 0)) {
        bool ok = true;
        std::vector<int> keep = conv_it;
        for (int i = 0; i < nprob; ++i) {
          ok = ok && keep[i] >= 0;
          if (from_cache) keep[i] = std::max(keep[i], cache_old[i]);
        }
        if (ok) g_pass_cache.put(skey, keep);
      }
      for (int i : order) {
        const unsigned long long* st = hst.data() + DL.lstat[i];
        const int nt = probs[i].nt;
        // bit patterns of non-negative doubles: at or above that of +inf means not finite
        constexpr unsigned long long kInf = 0x7ff0000000000000ull;
        unsigned long long res = 0, rho = 0;
        bool finite = true;
        for (int sg = 0; sg <= Si[i]; ++sg)
          for (int n = 0; n < nt; ++n) {
            const unsigned long long* q = st + ((size_t)sg * nt + n) * kStat;
            finite = finite && q[0] < kInf && q[1] < kInf && q[2] < kInf;
            rho = std::max(rho, q[2]);
            if (sg == Si[i]) {
              res = std::max(res, q[1]);
              h_lm[ofs_nt[i] + n] = val(q[0]);
            }
          }
        h_sc[4 * i] = finite ? val(res) : std::nan("");
        h_sc[4 * i + 1] = val(rho);
        h_sc[4 * i + 2] = std::nan("");
        if (stats) {
          // lane s formed the residual of U^(s) at every level from U^(s) of the level before:
          // its maxima are the Newton history inside the pass
          stats[i].schedule = PTS_SCHED_PIPELINE;
          stats[i].sweeps = kmax_all;
          stats[i].refine = 0;
          for (int sg = 1; sg < Si[i] && done[i] + sg < PTS_MAX_HIST; ++sg) {
            unsigned long long r = 0, g = 0;
            for (int n = 0; n < nt; ++n) {
              const unsigned long long* q = st + ((size_t)sg * nt + n) * kStat;
              r = std::max(r, q[1]);
              g = std::max(g, q[2]);
            }
            stats[i].res_inf[done[i] + sg] = val(r);
            stats[i].rho_max[done[i] + sg] = val(g);
            stats[i].upd_rms[done[i] + sg] = std::nan("");
          }
        }
        done[i] += Si[i];
      }
      if (prof) prof->collect(&pstat);
      was_pass = true;
      it += S - 1;
      continue;
    }
    if (use_mg) {
      // one Newton step: level after level, every lane-0 solver of the active instances; the
      // Chebyshev plans of every level from the current iterate's level maxima (host)
      std::vector<int> lanes;
      for (int i : order) lanes.push_back(i * kLanes);
      std::memset((void*)h_dd, 0, nlanes * sizeof(PcDesc));  // lanes 1.. stay inactive
      for (int i = 0; i < nprob; ++i) {
        h_dd[(size_t)i * kLanes] = lane_desc(i, 0);
        if (!active[i]) continue;
        int kmax_i = 0;
        for (int n = 0; n < probs[i].nt; ++n) {
          const int K = mg_cheb_plan(probs[i].mu_a, probs[i].mu_b, h_lm[ofs_nt[i] + n], lin_tol,
                                     h_cf + (ofs_nt[i] + n) * kMaxCheb);
          h_kt[ofs_nt[i] + n] = K;
          kmax_i = std::max(kmax_i, K);
        }
        const size_t q = (size_t)i * kLanes;
        HIPCHK(hipMemcpyAsync(mg_base + DL.K[q], h_kt + ofs_nt[i], (size_t)probs[i].nt * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(mg_base + DL.coef[q], h_cf + ofs_nt[i] * kMaxCheb,
                              (size_t)probs[i].nt * kMaxCheb * sizeof(float2), hipMemcpyHostToDevice, s));
        if (stats) {
          stats[i].sweeps = kmax_i;
          stats[i].refine = 0;
        }
      }
      std::vector<size_t> ce, od, ou;
      std::vector<std::vector<size_t>> cd, cu;
      if ((rc = build_items(lanes, ce, cd, cu, od, ou))) return rc;
      for (int n = 0; n < maxnt; ++n) {
        const int k = kpref[n];
        if (k == 0) continue;
        int kn = 0;  // iterations of level n: the most any instance in the prefix needs
        for (int q = 0; q < k; ++q) kn = std::max(kn, h_kt[ofs_nt[order[q]] + n]);
        for (int kk = 0; kk < kn; ++kk)
          vcycle(n, kk, true, (size_t)k, ce, cd, cu, od, ou, [&](int kind, int g) {
            double b = 0.0;
            for (int q = 0; q < k; ++q)
              if (kk < h_kt[ofs_nt[order[q]] + n]) b += kb(kind, order[q], kk, g, 8.0);
            return b;
          });
      }
    } else {
      // descriptors (inactive instances have no launches) and work items, longest first
      for (int i = 0; i < nprob; ++i) {
        BatchDesc& d = h_desc[i];
        std::memset(&d, 0, sizeof d);
        d.p = in[i].kp;
        d.g = in[i].g;
        d.U = U[i];
        d.R = in[i].R;
        d.dU = in[i].dU;
        d.Xs = in[i].Xs;
        d.rho = (const double*)in[i].rho;
        if (active[i]) {
          d.npacks = (int)std::min<size_t>(plans[i].packs.size(), kMaxPacks);
          d.sweeps = plans[i].sweeps;
          for (int l = 0; l < d.npacks; ++l) d.packs[l] = plans[i].packs[l];
        }
      }
      size_t nitems = 0;
      std::vector<size_t> cum(order.size() + 1, 0);
      std::vector<int> lmax(order.size() + 1, 0);
      for (size_t q = 0; q < order.size(); ++q) {
        const int i = order[q];
        for (int t = 0; t < ntiles[i]; ++t) h_items[nitems++] = make_int2(i, t);
        cum[q + 1] = nitems;
        lmax[q + 1] = std::max(lmax[q], h_desc[i].npacks);
      }
      HIPCHK(hipMemcpyAsync(d_desc, h_desc, (size_t)nprob * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(d_items, h_items, nitems * sizeof(int2), hipMemcpyHostToDevice, s));
      for (int n = 0; n < maxnt; ++n) {
        const int k = kpref[n];
        if (k == 0) continue;
        for (int l = 0; l < lmax[k]; ++l) {
          hipLaunchKernelGGL(kern, dim3((unsigned)cum[k]), dim3(kThreads), 0, s, d_desc, d_items, n, l);
          ++launches;
        }
      }
    }
    HIPCHK(hipGetLastError());
    for (int i : order) {
      const size_t count = (size_t)probs[i].nx * probs[i].ny * probs[i].nt;
      if (use_mg) prof_begin(prof, Prof::kKern + 6, s);
      hipLaunchKernelGGL(k_update, dim3(kUpdateBlocks), dim3(256), 0, s, count, U[i], in[i].dU, in[i].partial);
      hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, in[i].partial, kUpdateBlocks, in[i].rms);
      if (use_mg && prof) {  // read U, dU, write U
        prof->end(s);
        prof->recs.back().count = 2;
        prof->recs.back().bytes = 24.0 * (double)count;
      }
      launches += 2;
      if (use_mg) prof_begin(prof, Prof::kKern + 5, s);
      if ((rc = in[i].residual(U[i], u0[i], s, &launches))) return rc;
      if (use_mg && prof) {  // read U, write R
        prof->end(s);
        prof->recs.back().count = 3;
        prof->recs.back().bytes = 16.0 * (double)count;
      }
      if (use_mg) {
        prof_begin(prof, Prof::kKern + 7, s);
        level_max(i);
        if (prof) {
          prof->end(s);
          prof->recs.back().bytes = 8.0 * (double)count;
        }
      }
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_all(true, false, use_mg))) return rc;
    if (prof) prof->collect(&pstat);
  }
  if (stats)
    for (int i = 0; i < nprob; ++i) {
      stats[i].launches = launches;
      for (int j = 0; j < 8; ++j) {
        stats[i].kern_ms[j] = pstat.kern_ms[j];
        stats[i].kern_count[j] = pstat.kern_count[j];
        stats[i].kern_bytes[j] = pstat.kern_bytes[j];
      }
    }
  return worst;
}

// ---------------------------------------------------------------- batched wavefront
// Whether the instances are one problem with different initial conditions: same sizes,
// coefficients, precision and boundary data.
bool same_problem(const pts_problem* probs, int nprob) {
  const pts_problem& a = probs[0];
  for (int i = 1; i < nprob; ++i) {
    const pts_problem& b = probs[i];
    if (a.kind != b.kind || a.bc != b.bc || a.nx != b.nx || a.ny != b.ny || a.nt != b.nt ||
        a.precision != b.precision || a.hx != b.hx || a.hy != b.hy || a.dt != b.dt || a.mu_a != b.mu_a ||
        a.mu_b != b.mu_b || a.bdata != b.bdata || a.dt_levels != b.dt_levels)
      return false;
  }
  return true;
}

// Wavefront sequences over every instance at once: each anti-diagonal is one launch of
// grid (K stages x tiles, active instances), the per-instance arguments in the batch
// header. All instances run the same K per sequence (the plan follows the largest radius
// of the active instances); an instance leaves the batch once its residual meets tol.
// Returns PTS_ERR_INVALID_ARG with *fallback = true, before anything is written, when the
// inner solve does not fit the wavefront kernel.
int solve_wave_batched(const pts_problem* probs, int nprob, double* const* U, const double* const* u0, double tol,
                       int max_iter, char* header, char* wsb, const pts_options* o, pts_stats* stats,
                       hipStream_t s, bool* fallback, int* codes) {
  *fallback = false;
  const pts_problem* p = probs;
  for (int i = 0; i < nprob; ++i) codes[i] = PTS_OK;
  const bool use_graph = !o || o->use_graph != 0;
  // profiling: HIP events around each sequence (its replayed graph) on `s`; time / launches is
  // the mean launch interval of k_level_wave_batch
  Prof wprof;
  const bool profiling = o && o->profile;
  pts_stats wst;
  std::memset(&wst, 0, sizeof wst);
  const size_t ns = (size_t)p->nx * p->ny, st_count = ns * p->nt;
  std::vector<Instance> in(nprob);
  std::vector<char*> base(nprob);
  char* w = wsb;
  for (int i = 0; i < nprob; ++i) {
    base[i] = w;
    in[i].bind(probs + i, w);
    w += in[i].L.total;
    if (stats) std::memset(stats + i, 0, sizeof(pts_stats));
  }
  const Layout& L = in[0].L;
  // host staging: the arguments of the active instances, then per instance the two
  // residual scalars and the stage maxima of the last sequence
  const size_t s_sc = align_up((size_t)nprob * sizeof(WaveArgs));
  const size_t s_st = s_sc + align_up((size_t)nprob * 2 * 8);
  char* stage;
  int rc = host_stage(s_st + (size_t)nprob * (kMaxStages + 1) * 8, &stage);
  if (rc) return rc;
  WaveArgs* h_args = (WaveArgs*)stage;
  double* h_sc = (double*)(stage + s_sc);
  double* h_st = (double*)(stage + s_st);
  WaveArgs* d_args = (WaveArgs*)header;  // the bulk schedule's descriptor area (larger entries)
  static_assert(sizeof(WaveArgs) <= sizeof(BatchDesc), "batched wavefront arguments fit the header");
  int launches = 0;
  for (int i = 0; i < nprob; ++i) {
    HIPCHK(hipMemcpyAsync(base[i] + L.u0copy, u0[i], ns * 8, hipMemcpyDeviceToDevice, s));
    if ((rc = in[i].residual(U[i], u0[i], s, &launches, false))) return rc;
    HIPCHK(hipMemcpyAsync(h_sc + 2 * i, in[i].scal, 16, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  std::vector<char> active(nprob, 1);
  std::vector<int> needed(nprob, -1);
  int it = 0, worst = PTS_OK;
  Plan plan_used;
  auto drop = [&](int i, int err) {
    active[i] = 0;
    codes[i] = err;
    if (err && !worst) worst = err;
  };
  for (;;) {
    std::vector<int> act;
    double rho_all = 0.0;
    for (int i = 0; i < nprob; ++i) {
      if (!active[i]) continue;
      const double res = h_sc[2 * i], rhom = h_sc[2 * i + 1];
      pts_stats* st = stats ? stats + i : nullptr;
      if (st) {
        if (it < PTS_MAX_HIST) {
          st->res_inf[it] = res;
          st->rho_max[it] = rhom;
        }
        st->iterations = it;
        st->hist = std::min(it + 1, PTS_MAX_HIST);
        st->slab = p->nt;
        st->window = 1;
        st->schedule = PTS_SCHED_PIPELINE;
      }
      if (!std::isfinite(res) || !std::isfinite(rhom)) {
        drop(i, fail(PTS_ERR_NONFINITE, "instance %d: non-finite residual at Newton step %d", i, it));
      } else if (res <= tol) {
        if (needed[i] < 0) needed[i] = it;
        if (st) st->converged = 1;
        drop(i, PTS_OK);
      } else if (rhom >= 1.0) {
        drop(i, fail(PTS_ERR_NOT_DOMINANT, "instance %d: block not diagonally dominant (radius %.3g)", i, rhom));
      } else if (it >= max_iter) {
        drop(i, fail(PTS_ERR_NOT_CONVERGED, "instance %d: not converged after %d Newton steps (|R| = %.3e)", i,
                     it, res));
      } else {
        act.push_back(i);
        rho_all = std::max(rho_all, rhom);
      }
    }
    if (act.empty()) break;
    // inner plan and stage count as for one instance, from the batch entry of the problem
    // (else its one-instance entry) and the largest radius of the active instances
    Plan pl;
    int K = 1;
    const StageCache::E* ce = g_stage_cache.find(p, tol, ctag(o), 1);
    if (!ce) ce = g_stage_cache.find(p, tol, ctag(o), 0);
    if (!next_wave_plan(p, o, ce, rho_all, it, max_iter, &pl, &K)) {
      if (it == 0) {
        *fallback = true;
        return PTS_ERR_INVALID_ARG;
      }
      for (int i : act)
        drop(i, fail(PTS_ERR_NOT_DOMINANT, "instance %d: inner solve cannot reach the requested reduction", i));
      break;
    }
    const Geo g = in[0].g.whole ? in[0].g : geometry(p, wave_halo(pl));
    plan_used = pl;
    const int tl = tiles(p, g);
    const int nb = (int)act.size();
    for (int q = 0; q < nb; ++q) {
      const int i = act[q];
      if (stats) {
        stats[i].sweeps = pl.sweeps;
        stats[i].refine = pl.passes - 1;
      }
      double* res_part = (double*)(base[i] + L.res_part);
      hipLaunchKernelGGL(k_zero, dim3((unsigned)(((K + 1) * tl + 255) / 256)), dim3(256), 0, s,
                         (unsigned long long*)res_part, (K + 1) * tl);
      WaveArgs& wa = h_args[q];
      wa.Ur[0] = U[i];
      wa.Ur[1] = (double*)(base[i] + L.U1);
      wa.u0 = (const double*)(base[i] + L.u0copy);
      wa.rho_in = (const double*)in[i].rho;
      wa.rho_part = (double*)(base[i] + L.rho_part);
      wa.res_part = res_part;
      wa.tiles = tl;
      wa.stages = K;
    }
    launches += nb;
    HIPCHK(hipMemcpyAsync(d_args, h_args, (size_t)nb * sizeof(WaveArgs), hipMemcpyHostToDevice, s));
    const WaveBatchKernel kern = wave_batch_kernel(p, pl.fp32);
    const int ndiag = p->nt + 2 * (K - 1);
    auto launch_seq = [&](hipStream_t ls) -> int {
      for (int d = 0; d < ndiag; ++d)
        hipLaunchKernelGGL(kern, dim3((unsigned)(K * tl), (unsigned)nb), dim3(kThreads), 0, ls, in[0].kp,
                           (const WaveArgs*)d_args, g, d, pl.passes, pl.sweeps);
      HIPCHK(hipGetLastError());
      return PTS_OK;
    };
    if (profiling) wprof.begin(1, s);
    if (use_graph) {
      // the arguments are read from the header at run time: the key holds what the
      // launches themselves carry
      std::vector<char> key;
      const int extra[6] = {1, pl.passes, pl.sweeps, pl.fp32 ? 1 : 0, K, nb};
      key_append(key, in[0].kp, g, d_args, extra);
      rc = replay_or_capture(key, s, &launches, launch_seq);
    } else {
      rc = launch_seq(s);
      launches += ndiag;
    }
    if (profiling) {
      wprof.end(s);
      wprof.recs.back().count = ndiag;
      for (int d = 0; d < ndiag; ++d) wprof.bytes += nb * wave_bytes(p, K, d);
    }
    if (rc) return rc;
    for (int i : act) {
      double* res_st = (double*)(base[i] + L.res_st);
      hipLaunchKernelGGL(k_stage_max, dim3(K + 1), dim3(256), 0, s, (const double*)(base[i] + L.res_part), tl,
                         res_st);
      if (K & 1) HIPCHK(hipMemcpyAsync(U[i], base[i] + L.U1, st_count * 8, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h_st + (size_t)i * (kMaxStages + 1), res_st, (K + 1) * 8, hipMemcpyDeviceToHost, s));
    }
    launches += nb;
    HIPCHK(hipStreamSynchronize(s));
    // residuals of the iterates U_{it+1..it+K}; an instance still above tol gets the
    // all-level residual of U_{it+K} (the radii the next sequence starts from)
    bool again = false;
    for (int i : act) {
      const double* rs = h_st + (size_t)i * (kMaxStages + 1);
      bool bad = false;
      for (int k = 1; k <= K && !bad; ++k) {
        if (stats && it + k < PTS_MAX_HIST) stats[i].res_inf[it + k] = rs[k];
        if (rs[k] <= tol && needed[i] < 0) needed[i] = it + k;
        if (!std::isfinite(rs[k])) {
          if (stats) stats[i].iterations = it + k;
          drop(i, fail(PTS_ERR_NONFINITE, "instance %d: non-finite residual at Newton step %d", i, it + k));
          bad = true;
        }
      }
      if (bad) continue;
      if (rs[K] > tol) {
        if ((rc = in[i].residual(U[i], u0[i], s, &launches, false))) return rc;
        HIPCHK(hipMemcpyAsync(h_sc + 2 * i, in[i].scal, 16, hipMemcpyDeviceToHost, s));
        again = true;
      } else {
        h_sc[2 * i] = rs[K];
        h_sc[2 * i + 1] = 0.0;
      }
    }
    if (again) HIPCHK(hipStreamSynchronize(s));
    it += K;
  }
  // remember the largest step count any instance needed with this plan
  int most = -1;
  bool all = true;
  for (int i = 0; i < nprob; ++i) {
    most = std::max(most, needed[i]);
    all = all && needed[i] >= 0;
  }
  if (all && plan_used.sweeps > 0) {
    const StageCache::E* ce = g_stage_cache.find(p, tol, ctag(o), 1);
    if (!ce || (ce->sweeps == plan_used.sweeps && ce->passes == plan_used.passes) || ce->sweeps == 0)
      g_stage_cache.put(p, tol, ctag(o), plan_used.sweeps, plan_used.passes, std::max(most, 1), true, 1);
  }
  if (profiling) wprof.collect(&wst);
  if (stats)
    for (int i = 0; i < nprob; ++i) {
      stats[i].launches = launches;
      if (profiling) {
        stats[i].prof_ms[1] = wst.prof_ms[1];
        stats[i].prof_count[1] = wst.prof_count[1];
        stats[i].level_solve_bytes = wst.level_solve_bytes;
      }
    }
  return worst;
}

// Try inner plans on a batch of instances of one problem (each a full batched solve from the
// iterates in U, run twice: once to learn its Newton step count, once timed with HIP events)
// and cache the fastest for batches of this problem. U is restored on return (kept in each
// instance's residual array, which the wavefront schedule does not use).
int autotune_wave_batched(const pts_problem* probs, int nprob, double* const* U, const double* const* u0,
                          double tol, int max_iter, char* header, char* wsb, const pts_options* o, pts_stats* stats,
                          hipStream_t s) {
  const pts_problem* p = probs;
  const size_t bytes = (size_t)p->nx * p->ny * p->nt * 8, wb = layout(p).total;
  std::vector<double*> backup(nprob);
  for (int i = 0; i < nprob; ++i) {
    backup[i] = (double*)(wsb + (size_t)i * wb + layout(p).R);
    HIPCHK(hipMemcpyAsync(backup[i], U[i], bytes, hipMemcpyDeviceToDevice, s));
  }
  auto restore = [&]() -> int {
    for (int i = 0; i < nprob; ++i) HIPCHK(hipMemcpyAsync(U[i], backup[i], bytes, hipMemcpyDeviceToDevice, s));
    return PTS_OK;
  };
  const bool fp32 = p->precision == PTS_MIXED;
  std::vector<std::pair<int, int>> cands;
  if (!fp32) {
    for (int sw : {4, 5, 6, 7, 8, 10}) cands.push_back({sw, 1});
  } else {
    for (int sw : {3, 4, 5}) cands.push_back({sw, 2});
    for (int sw : {4, 5, 6, 8}) cands.push_back({sw, 1});
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best_sw = 0, best_pa = 0, best_steps = 0;
  pts_options o1 = o ? *o : pts_options{};
  o1.schedule = PTS_SCHED_PIPELINE;
  o1.profile = 0;
  o1.lin_tol = 0;
  o1.sweeps = 0;
  o1.refine = -1;  // the plan comes from the cache entry written for the candidate
  o1.stages = 0;
  std::vector<pts_stats> st(nprob);
  std::vector<int> codes(nprob);
  int rc = PTS_OK;
  for (auto& c : cands) {
    Plan probe;
    probe.sweeps = c.first;
    probe.passes = c.second;
    if (!geometry(p).whole && wave_halo(probe) > kMaxWaveHalo) continue;
    g_stage_cache.put(p, tol, ctag(o), c.first, c.second, 4, false, 1);
    bool fb = false, conv = true;
    for (int run = 0; run < 2 && conv; ++run) {
      if ((rc = restore())) break;
      if (run == 1) HIPCHK(hipEventRecord(e0, s));
      rc = solve_wave_batched(probs, nprob, U, u0, tol, max_iter, header, wsb, &o1, st.data(), s, &fb,
                              codes.data());
      if (run == 1) HIPCHK(hipEventRecord(e1, s));
      if (rc == PTS_ERR_HIP) break;
      for (int i = 0; i < nprob; ++i) conv = conv && st[i].converged;
      conv = conv && !fb;
    }
    if (rc == PTS_ERR_HIP) break;
    if (!conv) continue;
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      const StageCache::E* ce = g_stage_cache.find(p, tol, ctag(o), 1);
      best_ms = ms;
      best_sw = c.first;
      best_pa = c.second;
      best_steps = ce ? ce->steps : st[0].iterations;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int rr = restore();
  if (rc == PTS_ERR_HIP) return rc;
  if (rr) return rr;
  HIPCHK(hipStreamSynchronize(s));
  if (best_sw == 0) {
    g_stage_cache.put(p, tol, ctag(o), 0, 0, 0, false, 1);
    return fail(PTS_ERR_NOT_CONVERGED, "autotune: no wavefront plan converged on the batch");
  }
  g_stage_cache.put(p, tol, ctag(o), best_sw, best_pa, best_steps, false, 1);
  if (stats)
    for (int i = 0; i < nprob; ++i) {
      std::memset(stats + i, 0, sizeof(pts_stats));
      stats[i].sweeps = best_sw;
      stats[i].refine = best_pa - 1;
      stats[i].iterations = best_steps;
      stats[i].solve_ms = best_ms;
      stats[i].schedule = PTS_SCHED_PIPELINE;
      stats[i].slab = p->nt;
    }
  return PTS_OK;
}

// ------------------------------------------------ coarse-grid initial iterate (Section 4)
// A cubic spline is linear in its data: at a point s (in units of the node spacing) the spline
// through nodes z = 0..N-1 is sum_k w_k(s) y_k. The weights are formed here, column k being the
// spline through the k-th unit vector, and the kernels apply them along each axis.

// Tridiagonal solve with unit off-diagonals (Thomas): x = T^{-1} d, T = tridiag(1, diag, 1).
void thomas_unit(const std::vector<double>& diag, const std::vector<double>& d, std::vector<double>& x) {
  const size_t n = diag.size();
  std::vector<double> cp(n), dp(n);
  for (size_t i = 0; i < n; ++i) {
    const double den = diag[i] - (i ? cp[i - 1] : 0.0);
    cp[i] = 1.0 / den;
    dp[i] = (d[i] - (i ? dp[i - 1] : 0.0)) / den;
  }
  x.assign(n, 0.0);
  for (size_t i = n; i-- > 0;) x[i] = dp[i] - (i + 1 < n ? cp[i] * x[i + 1] : 0.0);
}

// Second derivatives M of the cubic spline through y at unit spacing: M_{z-1} + 4 M_z +
// M_{z+1} = 6 (y_{z-1} - 2 y_z + y_{z+1}) at the inner nodes, and either not-a-knot ends (one
// cubic across the first two and the last two intervals: M_0 - 2 M_1 + M_2 = 0 and likewise
// at the far end; substituted, the rows of nodes 1 and N-2 become 6 M_1 = d_1 and
// 6 M_{N-2} = d_{N-2}; N = 3 gives one parabola, N = 2 a line), or periodic (indices modulo N,
// N >= 3; the cyclic system by the Sherman-Morrison correction of a tridiagonal one).
void spline_second(const std::vector<double>& y, bool periodic, std::vector<double>& M) {
  const int N = (int)y.size();
  M.assign(N, 0.0);
  if (!periodic) {
    if (N < 3) return;
    const int n = N - 2;
    std::vector<double> d(n), sub(n, 1.0), diag(n, 4.0), sup(n, 1.0);
    for (int z = 1; z < N - 1; ++z) d[z - 1] = 6.0 * (y[z - 1] - 2.0 * y[z] + y[z + 1]);
    diag[0] = 6.0;
    sup[0] = 0.0;
    diag[n - 1] = 6.0;
    sub[n - 1] = 0.0;
    // Thomas with the modified end rows (sub[0] and sup[n-1] are outside the matrix)
    std::vector<double> cp(n), dp(n);
    for (int i = 0; i < n; ++i) {
      const double den = diag[i] - (i ? sub[i] * cp[i - 1] : 0.0);
      cp[i] = sup[i] / den;
      dp[i] = (d[i] - (i ? sub[i] * dp[i - 1] : 0.0)) / den;
    }
    for (int i = n - 1; i >= 0; --i) M[i + 1] = dp[i] - (i + 1 < n ? cp[i] * M[i + 2] : 0.0);
    M[0] = N == 3 ? M[1] : 2.0 * M[1] - M[2];
    M[N - 1] = N == 3 ? M[1] : 2.0 * M[N - 2] - M[N - 3];
    return;
  }
  // A = T + u v^T with corner entries 1: gamma = -4, T = A with diag[0] = 4 - gamma and
  // diag[N-1] = 4 - 1/gamma, u = (gamma, 0, .., 0, 1), v = (1, 0, .., 0, 1/gamma)
  const double gamma = -4.0;
  std::vector<double> diag(N, 4.0), d(N), u(N, 0.0), x, q;
  diag[0] = 4.0 - gamma;
  diag[N - 1] = 4.0 - 1.0 / gamma;
  for (int z = 0; z < N; ++z) d[z] = 6.0 * (y[(z + N - 1) % N] - 2.0 * y[z] + y[(z + 1) % N]);
  u[0] = gamma;
  u[N - 1] = 1.0;
  thomas_unit(diag, d, x);
  thomas_unit(diag, u, q);
  const double f = (x[0] + x[N - 1] / gamma) / (1.0 + q[0] + q[N - 1] / gamma);
  for (int z = 0; z < N; ++z) M[z] = x[z] - f * q[z];
}

// One axis of the interpolation as the kernels apply it: the second derivatives M = G y at
// the N spline nodes (column j of G: the M of the spline through the j-th unit vector), then at
// each fine point s_i (in node spacings) the value (1-t) y_z0 + t y_z1 + ((1-t)^3 - (1-t)) M_z0 / 6
// + (t^3 - t) M_z1 / 6 on its interval (z0, z1), t = s_i - z0.
struct AxisSpline {
  int N = 0;
  std::vector<double> G;    // [N][N]
  std::vector<int> zz;      // [nf][2]
  std::vector<double> w;    // [nf][4]
};
AxisSpline axis_spline(int N, bool periodic, const std::vector<double>& s) {
  AxisSpline A;
  A.N = N;
  A.G.assign((size_t)N * N, 0.0);
  std::vector<double> y(N), M;
  for (int j = 0; j < N; ++j) {
    y.assign(N, 0.0);
    y[j] = 1.0;
    spline_second(y, periodic, M);
    for (int k = 0; k < N; ++k) A.G[(size_t)k * N + j] = M[k];
  }
  for (double si : s) {
    int z0 = (int)std::floor(si);
    z0 = periodic ? ((z0 % N) + N) % N : std::max(0, std::min(z0, N - 2));
    const int z1 = periodic ? (z0 + 1) % N : z0 + 1;
    const double t = periodic ? si - std::floor(si) : si - z0, a = 1.0 - t;
    A.zz.push_back(z0);
    A.zz.push_back(z1);
    for (double v : {a, t, (a * a * a - a) / 6.0, (t * t * t - t) / 6.0}) A.w.push_back(v);
  }
  return A;
}

// The spline of a spatial axis with n fine and nc coarse nodes spanning the same domain:
// periodic (nodes = the coarse nodes, fine node i at i nc / n coarse spacings; i / cf where the
// grids nest), or Dirichlet (nodes: edge, the coarse nodes, edge; fine node i at
// (i + 1)(nc + 1) / (n + 1); (i + 1) / cf where they nest).
AxisSpline space_spline(bool periodic, int n, int nc) {
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i)
    s[i] = periodic ? (double)((long)i * nc) / n : (double)((long)(i + 1) * (nc + 1)) / (n + 1);
  return axis_spline(periodic ? nc : nc + 2, periodic, s);
}

// Device image of an AxisSpline for the kernels: G split into its inner columns [N][N - 2e]
// (e = 1 for an axis with edge nodes) and its edge columns, then the weights and intervals.
struct AxisDev {
  size_t g, glo, ghi, w, zz, total;
};
AxisDev axis_dev_layout(int N, int nf, bool edges) {
  AxisDev D;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  D.g = take((size_t)N * (N - (edges ? 2 : 0)) * 8);
  D.glo = take((size_t)N * 8);
  D.ghi = take((size_t)N * 8);
  D.w = take((size_t)nf * 32);
  D.zz = take((size_t)nf * 8);
  D.total = o;
  return D;
}
void axis_dev_fill(const AxisSpline& A, bool edges, const AxisDev& D, char* host) {
  const int N = A.N, nin = N - (edges ? 2 : 0), j0 = edges ? 1 : 0;
  double* g = (double*)(host + D.g);
  double* lo = (double*)(host + D.glo);
  double* hi = (double*)(host + D.ghi);
  for (int k = 0; k < N; ++k) {
    for (int j = 0; j < nin; ++j) g[(size_t)k * nin + j] = A.G[(size_t)k * N + j + j0];
    lo[k] = edges ? A.G[(size_t)k * N] : 0.0;
    hi[k] = edges ? A.G[(size_t)k * N + N - 1] : 0.0;
  }
  std::memcpy(host + D.w, A.w.data(), A.w.size() * 8);
  std::memcpy(host + D.zz, A.zz.data(), A.zz.size() * 4);
}

// The Thomas elimination of the not-a-knot spline through N evenly spaced nodes, as the
// k_spline_m_* kernels read it: the inner rows M_{z-1} + 4 M_z + M_{z+1} = d_z with the first
// and last reduced to 6 M = d; th[0..n): eliminated super-diagonal, th[n..2n): reciprocal
// pivots, n = N - 2.
void thomas_table(int N, double* th) {
  const int n = std::max(N - 2, 0);
  for (int k = 0; k < n; ++k) {
    const bool end = k == 0 || k == n - 1;
    const double sub = end ? 0.0 : 1.0, sup = k == 0 ? 0.0 : 1.0;
    const double den = (end ? 6.0 : 4.0) - (k ? sub * th[k - 1] : 0.0);
    th[k] = sup / den;
    th[n + k] = 1.0 / den;
  }
}

// The problem on the grid coarsened by cf in x, y and t (FP64 coarse solve). Where cf divides
// the grid (nx for periodic, nx + 1 for Dirichlet axes) the coarse nodes are every cf-th fine
// node; otherwise the coarse grid spans the same domain with nx / cf (periodic) or
// (nx + 1) / cf - 1 (Dirichlet) evenly spaced nodes. ceil(nt / cf) coarse levels of step
// cf dt (the last may end past the fine end time). Dirichlet data need nesting grids and levels.
int coarse_problem(const pts_problem* p, int cf, pts_problem* pc) {
  if (cf < 2) return fail(PTS_ERR_INVALID_ARG, "coarse iterate: cf must be >= 2");
  if (p->dt_levels) return fail(PTS_ERR_INVALID_ARG, "coarse iterate: uniform steps only (dt_levels is set)");
  *pc = *p;
  const bool per = p->bc == PTS_PERIODIC;
  auto axis = [&](int n, double h, int* nc, double* hc) -> bool {  // false: no coarse grid
    if (per) {
      *nc = n / cf;
      *hc = n % cf == 0 ? cf * h : n * h / *nc;
      return *nc >= 3;
    }
    *nc = (n + 1) / cf - 1;
    *hc = (n + 1) % cf == 0 ? cf * h : (n + 1) * h / (*nc + 1);
    return *nc >= 1;
  };
  if (!axis(p->nx, p->hx, &pc->nx, &pc->hx) || !axis(p->ny, p->hy, &pc->ny, &pc->hy))
    return fail(PTS_ERR_INVALID_ARG, "coarse iterate: cf leaves fewer than %s coarse nodes", per ? "3" : "1");
  const bool nested = p->nt % cf == 0 && (per ? p->nx % cf == 0 && p->ny % cf == 0
                                              : (p->nx + 1) % cf == 0 && (p->ny + 1) % cf == 0);
  if (p->bdata && !nested)
    return fail(PTS_ERR_INVALID_ARG, "coarse iterate: Dirichlet data need cf to divide nx + 1, ny + 1 and nt");
  pc->nt = (p->nt + cf - 1) / cf;
  pc->dt = cf * p->dt;
  pc->bdata = nullptr;
  pc->precision = PTS_FP64;
  return validate(pc);
}

// Workspace of the coarse start of nprob instances (each its own problem): the coarse solve's
// (one instance: pts_solve's; several: pts_solve_batched's), per instance the coarse iterate,
// u^0, Dirichlet data and spline tables, and the interpolation buffers the instances share
// (used one after another in stream order, sized for the largest).
struct CoarseInst {
  pts_problem pc;
  size_t Uc, u0c, Sx, Sy, St, Th, Thx, Thy, bdc, edges;  // Th*: Thomas tables of the t, x, y splines
  AxisDev dx, dy, dt;
};
struct CoarseLayout {
  size_t solver, tab, tab_end, T1, V, Mx, My, Mt, total;  // [tab, tab_end): every spline table
  std::vector<CoarseInst> in;
};
size_t coarse_solver_bytes(const std::vector<pts_problem>& pcs) {
  const int n = (int)pcs.size();
  if (n == 1) return layout(&pcs[0]).total;
  size_t t = batch_header_bytes(pcs.data(), n);
  for (const pts_problem& q : pcs) t += layout(&q).total;
  return t;
}
// rc: PTS_OK or the error of an instance's coarse problem
CoarseLayout coarse_layout(const pts_problem* p, int nprob, int cf, int* rc) {
  CoarseLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.in.resize(nprob);
  std::vector<pts_problem> pcs(nprob);
  *rc = PTS_OK;
  for (int i = 0; i < nprob && !*rc; ++i) {
    if ((*rc = validate(p + i))) break;
    *rc = coarse_problem(p + i, cf, &pcs[i]);
  }
  if (*rc) return L;
  L.solver = take(coarse_solver_bytes(pcs));
  L.tab = o;
  for (int i = 0; i < nprob; ++i) {
    const pts_problem& f = p[i];
    const pts_problem& c = pcs[i];
    CoarseInst& q = L.in[i];
    q.pc = c;
    const bool dir = f.bc != PTS_PERIODIC;
    q.dx = axis_dev_layout(c.nx + (dir ? 2 : 0), f.nx, dir);
    q.dy = axis_dev_layout(c.ny + (dir ? 2 : 0), f.ny, dir);
    q.dt = axis_dev_layout(c.nt + 1, f.nt, false);
    q.Sx = take(q.dx.total);
    q.Sy = take(q.dy.total);
    q.St = take(q.dt.total);
    q.Th = take((size_t)2 * (c.nt + 1) * 8);  // Thomas elimination of the time spline
    q.Thx = take((size_t)2 * (c.nx + 2) * 8);  // and of the Dirichlet x and y splines
    q.Thy = take((size_t)2 * (c.ny + 2) * 8);
  }
  L.tab_end = o;
  size_t t1 = 0, v = 0, mx = 0, my = 0, mt = 0;
  for (int i = 0; i < nprob; ++i) {
    const pts_problem& f = p[i];
    const pts_problem& c = pcs[i];
    CoarseInst& q = L.in[i];
    const bool dir = f.bc != PTS_PERIODIC;
    const size_t nsc = (size_t)c.nx * c.ny;
    const int Nx = c.nx + (dir ? 2 : 0), Ny = c.ny + (dir ? 2 : 0), Nt = c.nt + 1;
    q.Uc = take(nsc * c.nt * 8);
    q.u0c = take(nsc * 8);
    // Dirichlet data (the size does not depend on whether the caller passes any, so that a
    // workspace sized from the problem alone fits)
    q.bdc = take(dir ? (size_t)c.nt * 2 * (c.nx + c.ny) * 8 : 0);
    q.edges = take(dir ? (size_t)c.nt * 2 * (c.ny + f.nx) * 8 : 0);  // west_c, east_c, south_f, north_f
    t1 = std::max(t1, (size_t)c.nt * c.ny * f.nx);
    v = std::max(v, (size_t)c.nt * f.ny * f.nx);
    mx = std::max(mx, (size_t)c.nt * c.ny * Nx);  // second derivatives along each axis
    my = std::max(my, (size_t)c.nt * Ny * f.nx);
    mt = std::max(mt, (size_t)Nt * f.nx * f.ny);
  }
  L.T1 = take(t1 * 8);
  L.V = take(v * 8);
  L.Mx = take(mx * 8);
  L.My = take(my * 8);
  L.Mt = take(mt * 8);
  L.total = o;
  return L;
}

void launch_spline_eval(hipStream_t s, const char* tab, const AxisDev& D, int nf, int N, bool edges,
                        const double* in, long isa, long isk, long isb, int zoff, const double* in0,
                        const double* elo, const double* ehi, long esa, long esb, const double* M, long msa,
                        long msk, long msb, double* out, long osa, long osi, long osb, long na, long nb) {
  const long total = na * nf * nb;
  const unsigned blocks = (unsigned)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_spline_eval, dim3(blocks), dim3(256), 0, s, (const int2*)(tab + D.zz),
                     (const double4*)(tab + D.w), nf, N, edges ? 1 : 0, in, isa, isk, isb, zoff, in0, elo, ehi, esa,
                     esb, M, msa, msk, msb, out, osa, osi, osb, na, nb);
}

void launch_interp(hipStream_t s, const double* W, int nf, int nc, const double* in, long isa, long isk, long isb,
                   const double* in0, double* out, long osa, long osi, long osb, long na, long nb,
                   const double* Wlo = nullptr, const double* Whi = nullptr, const double* elo = nullptr,
                   const double* ehi = nullptr, long esa = 0, long esb = 0) {
  const long total = na * nf * nb;
  const unsigned blocks = (unsigned)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_interp_axis, dim3(blocks), dim3(256), 0, s, W, nf, nc, in, isa, isk, isb, in0, out, osa, osi,
                     osb, na, nb, Wlo, Whi, elo, ehi, esa, esb);
}

int no_judge(const pts_problem* p, const double* u0, double* U, void* solver_ws, int judge, int* chosen,
             double* res_pred, double* res_plain, hipStream_t s);

extern "C" {

const char* pts_last_error(void) { return g_err.c_str(); }

const char* pts_version(void) { return "pts 0.1 (gfx950)"; }

size_t pts_workspace_bytes(const pts_problem* p) {
  if (validate(p)) return 0;
  return layout(p).total;
}

int pts_window_bound(double h, double mu, double tau, double c, double eps, int wmax) {
  if (!(h > 0) || !(mu >= 0) || !(c > 0) || !(eps > 0) || wmax < 1)
    return fail(PTS_ERR_INVALID_ARG, "pts_window_bound: bad arguments");
  const double rhs = std::log(c * h * h * h * h / eps);
  int best = 0;
  for (int w = 1; w <= wmax; ++w) {
    const double t = tau > 0 ? tau : 1.0 / w;
    const double K = (1.0 + 8.0 * mu * t / (h * h)) / (1.0 + 2.0 * M_PI * M_PI * mu * t);
    if (w * std::log(K) < rhs)
      best = w;
    else
      break;
  }
  return best;
}

size_t pts_coarse_workspace_bytes(const pts_problem* p, int cf) { return pts_coarse_workspace_bytes_batched(p, 1, cf); }

size_t pts_coarse_workspace_bytes_batched(const pts_problem* probs, int nprob, int cf) {
  if (!probs || nprob < 1) {
    fail(PTS_ERR_INVALID_ARG, "coarse iterate: no instances");
    return 0;
  }
  int rc;
  const CoarseLayout L = coarse_layout(probs, nprob, cf, &rc);
  return rc ? 0 : L.total;
}

int pts_coarse_initial_iterate(const pts_problem* p, int cf, const double* u0, double* U, double tol, int max_iter,
                               void* workspace, size_t workspace_bytes, pts_stats* stats, pts_stream_t stream) {
  return pts_coarse_initial_iterate_batched(p, 1, cf, &u0, &U, tol, max_iter, workspace, workspace_bytes, stats,
                                            stream);
}

int pts_coarse_initial_iterate_batched(const pts_problem* probs, int nprob, int cf, const double* const* u0,
                                       double* const* U, double tol, int max_iter, void* workspace,
                                       size_t workspace_bytes, pts_stats* stats, pts_stream_t stream) {
  if (stats && nprob > 0) std::memset(stats, 0, (size_t)nprob * sizeof(pts_stats));
  if (!probs || nprob < 1) return fail(PTS_ERR_INVALID_ARG, "coarse iterate: no instances");
  int rc;
  const CoarseLayout L = coarse_layout(probs, nprob, cf, &rc);
  if (rc) return rc;
  for (int i = 1; i < nprob; ++i)
    if (probs[i].kind != probs[0].kind || probs[i].bc != probs[0].bc)
      return fail(PTS_ERR_INVALID_ARG, "coarse iterate: instance %d: kind and boundary kind differ", i);
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_coarse_initial_iterate: NULL array");
  for (int i = 0; i < nprob; ++i)
    if (!U[i] || !u0[i]) return fail(PTS_ERR_INVALID_ARG, "pts_coarse_initial_iterate: instance %d: NULL array", i);
  if (!(tol >= 0) || max_iter < 0) return fail(PTS_ERR_INVALID_ARG, "tol/max_iter");
  if (!workspace || workspace_bytes < L.total)
    return fail(PTS_ERR_WORKSPACE, "coarse workspace %zu bytes < required %zu", workspace_bytes, L.total);
  if ((uintptr_t)workspace % kAlign) return fail(PTS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  double* T1 = (double*)(w + L.T1);
  double* V = (double*)(w + L.V);
  double* Mx = (double*)(w + L.Mx);
  double* My = (double*)(w + L.My);
  double* Mt = (double*)(w + L.Mt);
  const bool per = probs[0].bc == PTS_PERIODIC, dir = !per;
  // spline tables of every instance: x and y (Dirichlet axes with edge nodes), time (nodes
  // t = m cf tau, m = 0..ceil(nt/cf); fine level n at (n + 1) / cf), and the Thomas
  // eliminations of the time spline's and the Dirichlet x and y splines' inner rows
  // (thomas_table); one upload
  {
    const size_t base = L.tab;
    std::vector<char> host(L.tab_end - base, 0);
    for (int i = 0; i < nprob; ++i) {
      const pts_problem& p = probs[i];
      const CoarseInst& q = L.in[i];
      const AxisSpline ax = space_spline(per, p.nx, q.pc.nx), ay = space_spline(per, p.ny, q.pc.ny);
      std::vector<double> stimes(p.nt);
      for (int n = 0; n < p.nt; ++n) stimes[n] = (double)(n + 1) / cf;
      const AxisSpline at = axis_spline(q.pc.nt + 1, false, stimes);
      axis_dev_fill(ax, dir, q.dx, host.data() + (q.Sx - base));
      axis_dev_fill(ay, dir, q.dy, host.data() + (q.Sy - base));
      axis_dev_fill(at, false, q.dt, host.data() + (q.St - base));
      thomas_table(q.pc.nt + 1, (double*)(host.data() + (q.Th - base)));
      thomas_table(q.pc.nx + 2, (double*)(host.data() + (q.Thx - base)));
      thomas_table(q.pc.ny + 2, (double*)(host.data() + (q.Thy - base)));
    }
    HIPCHK(hipMemcpyAsync(w + base, host.data(), host.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // pageable source: complete before it goes
  }
  // coarse u^0 (bilinear sampling; injection where the grids nest), Dirichlet data and the ends
  // of the spline lines, plain coarse iterates
  std::vector<double*> Uc(nprob), u0c(nprob);
  std::vector<pts_problem> pcs(nprob);
  for (int i = 0; i < nprob; ++i) {
    const pts_problem& p = probs[i];
    const CoarseInst& q = L.in[i];
    pcs[i] = q.pc;
    Uc[i] = (double*)(w + q.Uc);
    u0c[i] = (double*)(w + q.u0c);
    const size_t nsc = (size_t)q.pc.nx * q.pc.ny;
    if (dir && p.bdata) {
      double* west_c = (double*)(w + q.edges);
      double* east_c = west_c + (size_t)q.pc.nt * q.pc.ny;
      double* south_f = east_c + (size_t)q.pc.nt * q.pc.ny;
      double* north_f = south_f + (size_t)q.pc.nt * p.nx;
      const int count = q.pc.nt * (2 * (q.pc.nx + q.pc.ny) + 2 * p.nx);
      hipLaunchKernelGGL(k_cf_bdata, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p.bdata, p.nx, p.ny,
                         q.pc.nx, q.pc.ny, cf, q.pc.nt, (double*)(w + q.bdc), west_c, east_c, south_f, north_f);
      pcs[i].bdata = (const double*)(w + q.bdc);
    }
    hipLaunchKernelGGL(k_cf_sample, dim3((unsigned)((nsc + 255) / 256)), dim3(256), 0, s, u0[i], p.nx, p.ny,
                       q.pc.nx, q.pc.ny, per ? 1 : 0, u0c[i]);
    const unsigned bb = (unsigned)std::min<size_t>((nsc * q.pc.nt + 255) / 256, 8192);
    hipLaunchKernelGGL(k_broadcast, dim3(bb), dim3(256), 0, s, nsc, q.pc.nt, Uc[i], (const double*)u0c[i]);
  }
  HIPCHK(hipGetLastError());
  // the coarse solves (all-at-once Newton: by Theorem 1 the root is the sequential coarse
  // solution); several instances share batched launches
  if (nprob == 1)
    rc = solve_slabs(&pcs[0], Uc[0], u0c[0], tol, max_iter, w + L.solver, nullptr, stats, s);
  else
    rc = pts_solve_batched(pcs.data(), nprob, Uc.data(), (const double* const*)u0c.data(), tol, max_iter,
                           w + L.solver, coarse_solver_bytes(pcs), nullptr, stats, stream);
  if (rc) return rc;
  // splines per instance, each as second derivatives then evaluation: x (coarse rows ->
  // T1[m][yc][x]), y (-> V[m][y][x]), t (u^0 and V -> U[n]); x lines of row yc at level m end in
  // west_c/east_c[m][yc], y lines of column x in south_f/north_f[m][x]. The instances reuse the
  // buffers in stream order.
  for (int i = 0; i < nprob; ++i) {
    const pts_problem& p = probs[i];
    const CoarseInst& q = L.in[i];
    const pts_problem& pc = q.pc;
    const char* Sx = w + q.Sx;
    const char* Sy = w + q.Sy;
    const char* St = w + q.St;
    const double *west_c = nullptr, *east_c = nullptr, *south_f = nullptr, *north_f = nullptr;
    if (dir && p.bdata) {
      west_c = (const double*)(w + q.edges);
      east_c = west_c + (size_t)pc.nt * pc.ny;
      south_f = east_c + (size_t)pc.nt * pc.ny;
      north_f = south_f + (size_t)pc.nt * p.nx;
    }
    const long nx = p.nx, ns = nx * p.ny;
    const int Nx = pc.nx + (dir ? 2 : 0), Ny = pc.ny + (dir ? 2 : 0), Nt = pc.nt + 1, zoff = dir ? 1 : 0;
    const long nax = (long)pc.nt * pc.ny;
    // second derivatives along x: a tridiagonal solve per Dirichlet line, the dense weights of the
    // periodic spline otherwise
    const unsigned lbx = (unsigned)std::min<long>((nax + 255) / 256, 65536);
    if (dir)
      hipLaunchKernelGGL(k_spline_m_line, dim3(lbx), dim3(256), 0, s, (const double*)(w + q.Thx), Nx,
                         (const double*)Uc[i], (long)pc.nx, 1L, 0L, west_c, east_c, 1L, 0L, Mx, (long)Nx, 1L, 0L, nax,
                         1L);
    else
      launch_interp(s, (const double*)(Sx + q.dx.g), Nx, pc.nx, Uc[i], pc.nx, 1, 0, nullptr, Mx, Nx, 1, 0, nax, 1,
                    nullptr, (const double*)(Sx + q.dx.ghi), west_c, east_c, 1, 0);
    launch_spline_eval(s, Sx, q.dx, p.nx, Nx, dir, Uc[i], pc.nx, 1, 0, zoff, nullptr, west_c, east_c, 1, 0, Mx, Nx,
                       1, 0, T1, nx, 1, 0, nax, 1);
    const unsigned lby = (unsigned)std::min<long>(((long)pc.nt * nx + 255) / 256, 65536);
    if (dir)
      hipLaunchKernelGGL(k_spline_m_line, dim3(lby), dim3(256), 0, s, (const double*)(w + q.Thy), Ny,
                         (const double*)T1, (long)pc.ny * nx, nx, 1L, south_f, north_f, nx, 1L, My, (long)Ny * nx, nx,
                         1L, (long)pc.nt, nx);
    else
      launch_interp(s, (const double*)(Sy + q.dy.g), Ny, pc.ny, T1, (long)pc.ny * nx, nx, 1, nullptr, My,
                    (long)Ny * nx, nx, 1, pc.nt, nx, nullptr, (const double*)(Sy + q.dy.ghi), south_f, north_f, nx, 1);
    launch_spline_eval(s, Sy, q.dy, p.ny, Ny, dir, T1, (long)pc.ny * nx, nx, 1, zoff, nullptr, south_f, north_f,
                       nx, 1, My, (long)Ny * nx, nx, 1, V, ns, nx, 1, pc.nt, nx);
    hipLaunchKernelGGL(k_spline_m_time, dim3((unsigned)std::min<long>((ns + 255) / 256, 65536)), dim3(256), 0, s,
                       (const double*)(w + q.Th), Nt, u0[i], (const double*)V, ns, Mt);
    const int run = std::max(kSplineRun, (p.nt + 65534) / 65535);
    hipLaunchKernelGGL(k_spline_eval_time,
                       dim3((unsigned)std::min<long>((ns + 255) / 256, 65536), (unsigned)((p.nt + run - 1) / run)),
                       dim3(256), 0, s, (const int2*)(St + q.dt.zz), (const double4*)(St + q.dt.w), p.nt, run, u0[i],
                       (const double*)V, ns, (const double*)Mt, U[i]);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return PTS_OK;
}

int pts_init_plain(const pts_problem* p, double* U, const double* u0, pts_stream_t stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_init_plain: NULL array");
  const size_t ns = (size_t)p->nx * p->ny;
  const size_t total = ns * p->nt;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_broadcast, dim3(blocks), dim3(256), 0, (hipStream_t)stream, ns, p->nt, U, u0);
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

int pts_assemble(const pts_problem* p, const double* U, const double* u0, double* R, double* coef, double* res_inf,
                 pts_stream_t stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!U || !u0 || !R) return fail(PTS_ERR_INVALID_ARG, "pts_assemble: NULL array");
  hipStream_t s = (hipStream_t)stream;
  KProb kp = kprob(p);
  const int tilesx = (p->nx + 63) / 64, tilesy = (p->ny + kResRows - 1) / kResRows;
  dim3 grid((unsigned)(tilesx * tilesy), (unsigned)p->nt);
  hipLaunchKernelGGL(residual_kernel(p), grid, dim3(256), 0, s, kp, U, u0, R, coef, nullptr);
  HIPCHK(hipGetLastError());
  if (res_inf) {
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, R, (size_t)p->nx * p->ny * p->nt,
                       (unsigned long long*)res_inf);
    HIPCHK(hipGetLastError());
  }
  return PTS_OK;
}

int pts_newton_step(const pts_problem* p, double* U, const double* u0, void* workspace, size_t workspace_bytes,
                    const pts_options* opts, pts_stats* stats, pts_stream_t stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  int rc = validate(p);
  if (!rc) rc = check_opts(opts);
  if (!rc) rc = check_ws(p, workspace, workspace_bytes);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_newton_step: NULL array");
  double* hs;
  bool cplx = false;
  rc = host_scalars(&hs);
  if (!rc) rc = convection_flag(p, u0, workspace, (hipStream_t)stream, hs, &cplx);
  if (rc) return rc;
  return solve_bulk(p, U, u0, 0.0, 1, workspace, opts, stats, (hipStream_t)stream, true, cplx);
}

int pts_newton_step_static(const pts_problem* p, double* U, const double* u0, const pts_options* opts,
                           pts_stats* stats, pts_stream_t stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  int rc = validate(p);
  if (!rc) rc = check_opts(opts);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_newton_step_static: NULL array");
  if (opts && opts->profile)
    return fail(PTS_ERR_INVALID_ARG, "pts_newton_step_static: profiling creates events; not available here");
  const size_t need = layout(p).total;
  if (need > kStaticScratchBytes)
    return fail(PTS_ERR_WORKSPACE, "pts_newton_step_static: problem needs %zu bytes of scratch, the static "
                "scratch holds %zu", need, kStaticScratchBytes);
  void* ws = nullptr;
  rc = static_scratch(&ws);
  if (rc) return rc;
  double hs[4] = {0.0, 0.0, 0.0, 0.0};
  bool cplx = false;
  rc = convection_flag(p, u0, ws, (hipStream_t)stream, hs, &cplx);
  if (rc) return rc;
  return solve_bulk(p, U, u0, 0.0, 1, ws, opts, stats, (hipStream_t)stream, true, cplx, hs);
}

size_t pts_products_workspace_bytes(const pts_problem* p) {
  if (prod_check(p)) return 0;
  const ProdLayout L = prod_layout(p);
  if ((L.total - L.band) / 8 > 0x7fffffffull) {
    fail(PTS_ERR_INVALID_ARG, "explicit products: the bands exceed 2^31 words");
    return 0;
  }
  return L.total;
}

}  // extern "C"

namespace {
int prod_args(const pts_problem* p, const double* U, const double* u0, void* ws, size_t bytes) {
  int rc = prod_check(p);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "explicit products: NULL array");
  const size_t need = pts_products_workspace_bytes(p);
  if (need == 0) return PTS_ERR_INVALID_ARG;
  if (!ws || bytes < need) return fail(PTS_ERR_WORKSPACE, "explicit products: workspace %zu < %zu bytes", bytes, need);
  if ((uintptr_t)ws % kAlign) return fail(PTS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return PTS_OK;
}
}  // namespace

extern "C" {

int pts_newton_step_products(const pts_problem* p, double* U, const double* u0, void* workspace,
                             size_t workspace_bytes, pts_stats* stats, pts_stream_t stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  int rc = prod_args(p, U, u0, workspace, workspace_bytes);
  if (rc) return rc;
  double* hs;
  if ((rc = host_scalars(&hs))) return rc;
  const ProdLayout L = prod_layout(p);
  rc = prod_step(p, U, u0, (char*)workspace, L, stats, 0, (hipStream_t)stream, hs);
  if (stats) {
    stats->iterations = 1;
    stats->hist = 1;
    stats->window = p->nt;
    stats->schedule = PTS_SCHED_BULK;
  }
  return rc;
}

int pts_solve_products(const pts_problem* p, double* U, const double* u0, double tol, int max_iter,
                       void* workspace, size_t workspace_bytes, pts_stats* stats, pts_stream_t stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  int rc = prod_args(p, U, u0, workspace, workspace_bytes);
  if (rc) return rc;
  if (!(tol >= 0) || max_iter < 0) return fail(PTS_ERR_INVALID_ARG, "tol/max_iter");
  hipStream_t s = (hipStream_t)stream;
  double* hs;
  if ((rc = host_scalars(&hs))) return rc;
  const ProdLayout L = prod_layout(p);
  char* ws = (char*)workspace;
  const auto t0 = std::chrono::steady_clock::now();
  int it = 0;
  for (;; ++it) {
    // max |R| of the current iterate
    rc = launch_residual(p, kprob(p), U, u0, nullptr, nullptr, (unsigned long long*)(ws + L.lvl),
                         (unsigned long long*)(ws + L.scal), s);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(hs, ws + L.scal, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats && it < PTS_MAX_HIST) stats->res_inf[it] = hs[0];
    if (stats) {
      stats->iterations = it;
      stats->hist = std::min(it + 1, PTS_MAX_HIST);
      stats->window = p->nt;
      stats->schedule = PTS_SCHED_BULK;
    }
    if (!std::isfinite(hs[0])) return fail(PTS_ERR_NONFINITE, "explicit products: non-finite residual at step %d", it);
    if (hs[0] <= tol) {
      if (stats) stats->converged = 1;
      break;
    }
    if (it >= max_iter) return fail(PTS_ERR_NOT_CONVERGED, "explicit products: not converged after %d steps", it);
    if ((rc = prod_step(p, U, u0, ws, L, stats, it, s, hs))) return rc;
  }
  if (stats)
    stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return PTS_OK;
}

int pts_product_diamond(const pts_problem* p, const double* U, const double* u0, int n, double* out,
                        void* workspace, size_t workspace_bytes, pts_stream_t stream) {
  int rc = prod_args(p, U, u0, workspace, workspace_bytes);
  if (rc) return rc;
  if (n < 1 || n > p->nt || !out) return fail(PTS_ERR_INVALID_ARG, "pts_product_diamond: level %d", n);
  const ProdLayout L = prod_layout(p);
  const double* last = nullptr;
  rc = prod_products(p, L, (char*)workspace, U, u0, n, false, (hipStream_t)stream, &last);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, last, (size_t)dia_count(n) * p->nx * p->ny * 8, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return PTS_OK;
}

int pts_solve(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* workspace,
              size_t workspace_bytes, const pts_options* opts, pts_stats* stats, pts_stream_t stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  int rc = validate(p);
  if (!rc) rc = check_opts(opts);
  if (!rc) rc = check_ws(p, workspace, workspace_bytes);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_solve: NULL array");
  if (!(tol >= 0) || max_iter < 0) return fail(PTS_ERR_INVALID_ARG, "tol/max_iter");
  const auto t0 = std::chrono::steady_clock::now();
  rc = solve_slabs(p, U, u0, tol, max_iter, workspace, opts, stats, (hipStream_t)stream);
  if (stats)
    stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int pts_autotune(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* workspace,
                 size_t workspace_bytes, const pts_options* opts, pts_stats* stats, pts_stream_t stream) {
  int rc = validate(p);
  if (!rc) rc = check_opts(opts);
  if (!rc) rc = check_ws(p, workspace, workspace_bytes);
  if (rc) return rc;
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_autotune: NULL array");
  if (p->dt_levels)
    return fail(PTS_ERR_INVALID_ARG, "pts_autotune tunes the wavefront schedule, which takes uniform steps");
  hipStream_t s = (hipStream_t)stream;
  const size_t ns = (size_t)p->nx * p->ny;
  const size_t bytes = ns * p->nt * 8;
  // U is kept in a temporary device copy while trial solves overwrite it (the only
  // allocation the library makes, freed before returning)
  double* backup = nullptr;
  HIPCHK(hipMalloc((void**)&backup, bytes));
  struct Free {
    double* b;
    ~Free() { (void)hipFree(b); }
  } guard{backup};
  HIPCHK(hipMemcpyAsync(backup, U, bytes, hipMemcpyDeviceToDevice, s));
  // slab length first: one safeguarded solve from the given iterate
  if (g_slab_cache.get(p) >= p->nt) {
    pts_stats st0;
    rc = solve_slabs(p, U, u0, tol, max_iter, workspace, opts, &st0, s);
    HIPCHK(hipMemcpyAsync(U, backup, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (rc) return rc;
  }
  const int L = g_slab_cache.get(p);
  if (L >= p->nt) {
    rc = autotune_wave(p, U, u0, tol, max_iter, workspace, opts, stats, s);
  } else {
    // tune the inner plan on the first slab, from its plain iterate
    pts_problem sub = *p;
    sub.nt = L;
    const size_t total = ns * L;
    const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_broadcast, dim3(blocks), dim3(256), 0, s, ns, L, U, u0);
    HIPCHK(hipGetLastError());
    rc = autotune_wave(&sub, U, u0, tol, max_iter, workspace, opts, stats, s);
    if (stats) stats->slab = L;
  }
  HIPCHK(hipMemcpyAsync(U, backup, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int pts_no_initial_iterate(const pts_problem* p, const pts_no_config* cfg, const float* params, const double* u0,
                           double* U, void* no_ws, size_t no_ws_bytes, void* solver_ws, size_t solver_ws_bytes,
                           int judge, int* chosen, double* res_pred, double* res_plain, pts_stream_t stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!cfg || p->bc != PTS_PERIODIC || cfg->nx != p->nx || cfg->ny != p->ny || cfg->nt != p->nt)
    return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate: network and problem disagree");
  if (p->dt_levels) return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate: uniform steps only");
  if (judge != PTS_NO_JUDGE_RESIDUAL && judge != PTS_NO_JUDGE_ACCUMULATED)
    return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate: judge %d", judge);
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate: NULL array");
  if ((rc = check_ws(p, solver_ws, solver_ws_bytes))) return rc;
  rc = pts_no_forward(cfg, params, u0, U, no_ws, no_ws_bytes, stream);
  if (rc) return rc;
  return no_judge(p, u0, U, solver_ws, judge, chosen, res_pred, res_plain, (hipStream_t)stream);
}

int pts_no_initial_iterate_batched(const pts_problem* p, const pts_no_config* cfg, const float* params, int batch,
                                   const double* const* u0, double* const* U, void* no_ws, size_t no_ws_bytes,
                                   void* solver_ws, size_t solver_ws_bytes, int judge, int* chosen,
                                   pts_stream_t stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!cfg || p->bc != PTS_PERIODIC || cfg->nx != p->nx || cfg->ny != p->ny || cfg->nt != p->nt)
    return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate_batched: network and problem disagree");
  if (p->dt_levels) return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate_batched: uniform steps only");
  if (judge != PTS_NO_JUDGE_RESIDUAL && judge != PTS_NO_JUDGE_ACCUMULATED)
    return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate_batched: judge %d", judge);
  if (batch < 1 || !U || !u0) return fail(PTS_ERR_INVALID_ARG, "pts_no_initial_iterate_batched: NULL array");
  if ((rc = check_ws(p, solver_ws, solver_ws_bytes))) return rc;
  rc = pts_no_forward_batched(cfg, params, batch, u0, U, no_ws, no_ws_bytes, stream);
  if (rc) return rc;
  for (int b = 0; b < batch; ++b)
    if ((rc = no_judge(p, u0[b], U[b], solver_ws, judge, chosen ? chosen + b : nullptr, nullptr, nullptr,
                       (hipStream_t)stream)))
      return rc;
  return PTS_OK;
}

}  // extern "C"

// The judge of a predicted iterate in U against the plain one (see pts_no_initial_iterate):
// U keeps the prediction or becomes the plain iterate.
int no_judge(const pts_problem* p, const double* u0, double* U, void* solver_ws, int judge, int* chosen,
             double* res_pred, double* res_plain, hipStream_t s) {
  int rc;
  Instance in;
  in.bind(p, solver_ws);
  int dummy = 0;
  const size_t ns = (size_t)p->nx * p->ny;
  const bool acc = judge == PTS_NO_JUDGE_ACCUMULATED;
  // residual of the prediction in the judge's norm -> scal[0]
  const int nchunks = (p->nt + kJudgeLevels - 1) / kJudgeLevels;
  if (acc && 3 * nchunks <= p->nt) {
    // accumulated form in two passes over U; the residual buffer (nt levels) holds the three
    // chunk summaries
    double* tot = in.R;
    double* hi = tot + (size_t)nchunks * ns;
    double* lo = hi + (size_t)nchunks * ns;
    const dim3 g1((unsigned)((ns + 255) / 256), (unsigned)nchunks);
    hipLaunchKernelGGL(k_judge_chunks<1>, g1, dim3(256), 0, s, in.kp, U, u0, tot, hi, lo);
    const unsigned blocks = (unsigned)std::min<size_t>((ns + 255) / 256, kUpdateBlocks);
    hipLaunchKernelGGL(k_judge_fold, dim3(blocks), dim3(256), 0, s, ns, nchunks, tot, hi, lo, in.partial);
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, in.partial, (size_t)blocks, in.scal);
  } else {
    // stored residual (nt < 3 leaves no room for the summaries), accumulated if asked
    if ((rc = in.residual(U, u0, s, &dummy, acc))) return rc;
    if (acc) {
      const unsigned blocks = (unsigned)std::min<size_t>((ns + 63) / 64, kUpdateBlocks);
      hipLaunchKernelGGL(k_cumsum_absmax, dim3(blocks), dim3(64), 0, s, ns, p->nt, in.R, in.partial);
      hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, in.partial, (size_t)blocks, in.scal);
    }
  }
  // the plain iterate's residual is -tau F(u^0) at every level (u^n - u^{n-1} = 0), i.e. the
  // one-level residual at u^0 (-> scal[2]); its accumulated form at level n is n times that
  pts_problem one = *p;
  one.nt = 1;
  if ((rc = launch_residual(&one, kprob(&one), u0, u0, nullptr, nullptr, in.rho, in.scal + 2, s))) return rc;
  const double mult = acc ? (double)p->nt : 1.0;
  const unsigned blocks = (unsigned)std::min<size_t>((ns * p->nt + 255) / 256, 8192);
  hipLaunchKernelGGL(k_judge_apply, dim3(blocks), dim3(256), 0, s, ns, p->nt, U, u0, in.scal, mult);
  HIPCHK(hipGetLastError());
  if (chosen || res_pred || res_plain) {
    double* hs;
    if ((rc = host_scalars(&hs))) return rc;
    HIPCHK(hipMemcpyAsync(hs, in.scal, 4 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rp = hs[0], r0 = hs[2] * mult;
    if (chosen) *chosen = (std::isfinite(rp) && rp < r0) ? 1 : 0;
    if (res_pred) *res_pred = rp;
    if (res_plain) *res_plain = r0;
  }
  return PTS_OK;
}

extern "C" {

size_t pts_workspace_bytes_batched(const pts_problem* probs, int nprob) {
  if (!probs || nprob < 1) {
    fail(PTS_ERR_INVALID_ARG, "no problems");
    return 0;
  }
  size_t t = 0;
  for (int i = 0; i < nprob; ++i) {
    if (validate(probs + i)) return 0;
    t += layout(probs + i).total;
  }
  return batch_header_bytes(probs, nprob) + t;
}

int pts_solve_batched(const pts_problem* probs, int nprob, double* const* U, const double* const* u0, double tol,
                      int max_iter, void* workspace, size_t workspace_bytes, const pts_options* opts,
                      pts_stats* stats, pts_stream_t stream) {
  const size_t need = pts_workspace_bytes_batched(probs, nprob);
  if (need == 0) return PTS_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < need) return fail(PTS_ERR_WORKSPACE, "batched workspace too small");
  if ((uintptr_t)workspace % kAlign) return fail(PTS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "NULL array list");
  for (int i = 0; i < nprob; ++i)
    if (!U[i] || !u0[i]) return fail(PTS_ERR_INVALID_ARG, "instance %d: NULL array", i);
  int rc = check_opts(opts);
  if (rc) return rc;
  if (!(tol >= 0) || max_iter < 0) return fail(PTS_ERR_INVALID_ARG, "tol/max_iter");
  bool uniform = true;
  for (int i = 1; i < nprob; ++i)
    uniform = uniform && probs[i].bc == probs[0].bc && probs[i].precision == probs[0].precision;
  const int sched = opts ? opts->schedule : PTS_SCHED_AUTO;
  char* w = (char*)workspace + batch_header_bytes(probs, nprob);
  // one problem with different initial conditions: batched wavefront sequences
  if (same_problem(probs, nprob) && sched != PTS_SCHED_BULK && !probs[0].dt_levels &&
      !(opts && (opts->window > 1 || opts->wave_launch == 1)) &&
      g_slab_cache.get(probs) >= probs[0].nt) {
    std::vector<int> codes(nprob);
    bool fb = false;
    rc = solve_wave_batched(probs, nprob, U, u0, tol, max_iter, (char*)workspace, w, opts, stats,
                            (hipStream_t)stream, &fb, codes.data());
    if (!fb) {
      // an instance whose Newton iteration diverged from its given iterate is solved alone,
      // with the slab safeguard of pts_solve (from the plain iterate of each slab)
      int worst = PTS_OK;
      const size_t b = layout(probs).total;
      for (int i = 0; i < nprob; ++i) {
        int r = codes[i];
        if (r == PTS_ERR_NONFINITE || r == PTS_ERR_SINGULAR || r == PTS_ERR_NOT_DOMINANT) {
          pts_stats one;
          pts_stats* sp = stats ? stats + i : &one;
          std::memset(sp, 0, sizeof *sp);
          r = solve_slabs(probs + i, U[i], u0[i], tol, max_iter, w + (size_t)i * b, opts, sp, (hipStream_t)stream);
        }
        if (r && !worst) worst = r;
      }
      return rc == PTS_ERR_HIP ? rc : worst;
    }
    if (sched == PTS_SCHED_PIPELINE) return fail(PTS_ERR_INVALID_ARG, "the inner solve does not fit the wavefront schedule");
  }
  const bool shared = uniform && !(opts && (opts->schedule == PTS_SCHED_PIPELINE || opts->window > 1));
  if (shared) return solve_batched_bulk(probs, nprob, U, u0, tol, max_iter, (char*)workspace, w, opts, stats,
                                        (hipStream_t)stream);
  // one instance after another (mixed boundary kinds or precisions, the wavefront schedule,
  // Theorem-1 windows)
  int worst = PTS_OK;
  for (int i = 0; i < nprob; ++i) {
    const size_t b = layout(probs + i).total;
    int r = pts_solve(probs + i, U[i], u0[i], tol, max_iter, w, b, opts, stats ? stats + i : nullptr, stream);
    if (r && !worst) worst = r;
    w += b;
  }
  return worst;
}

int pts_autotune_batched(const pts_problem* probs, int nprob, double* const* U, const double* const* u0, double tol,
                         int max_iter, void* workspace, size_t workspace_bytes, const pts_options* opts,
                         pts_stats* stats, pts_stream_t stream) {
  const size_t need = pts_workspace_bytes_batched(probs, nprob);
  if (need == 0) return PTS_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < need) return fail(PTS_ERR_WORKSPACE, "batched workspace too small");
  if ((uintptr_t)workspace % kAlign) return fail(PTS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (!U || !u0) return fail(PTS_ERR_INVALID_ARG, "NULL array list");
  for (int i = 0; i < nprob; ++i)
    if (!U[i] || !u0[i]) return fail(PTS_ERR_INVALID_ARG, "instance %d: NULL array", i);
  int rc = check_opts(opts);
  if (rc) return rc;
  if (!(tol >= 0) || max_iter < 0) return fail(PTS_ERR_INVALID_ARG, "tol/max_iter");
  if (!same_problem(probs, nprob))
    return fail(PTS_ERR_INVALID_ARG, "pts_autotune_batched: the instances are not one problem");
  char* w = (char*)workspace + batch_header_bytes(probs, nprob);
  return autotune_wave_batched(probs, nprob, U, u0, tol, max_iter, (char*)workspace, w, opts, stats,
                               (hipStream_t)stream);
}

}  // extern "C"
