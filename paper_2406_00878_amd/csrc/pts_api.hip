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
#include <string>
#include <vector>

#include "../../include/pts.h"
#include "pts_kernels.hip"

using namespace pts;

namespace {

thread_local std::string g_err = "no error";

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

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int validate(const pts_problem* p) {
  if (!p) return fail(PTS_ERR_INVALID_ARG, "problem is NULL");
  if (p->kind != PTS_HEAT && p->kind != PTS_BURGERS) return fail(PTS_ERR_INVALID_ARG, "kind %d", p->kind);
  if (p->bc != PTS_DIRICHLET && p->bc != PTS_PERIODIC) return fail(PTS_ERR_INVALID_ARG, "bc %d", p->bc);
  if (p->nx < 1 || p->ny < 1 || p->nt < 1) return fail(PTS_ERR_INVALID_ARG, "sizes %d x %d x %d", p->nx, p->ny, p->nt);
  if ((long long)p->nx * p->ny > (1ll << 30)) return fail(PTS_ERR_INVALID_ARG, "level too large");
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
  return k;
}

// Workspace layout of one instance.
struct Layout {
  size_t R, dU, Xs, rho, scal, partial, rms, total;
};

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
  L.total = o;
  return L;
}

Geo geometry(const pts_problem* p) {
  Geo g;
  if (p->bc == PTS_DIRICHLET && p->nx <= 64 && p->ny <= 64) {
    g.whole = 1;
    g.H = 0;
    g.TX = 64;
    g.TY = 64;
    g.tilesx = 1;
  } else {
    g.whole = 0;
    g.H = kHalo;
    g.TX = 64 - 2 * kHalo;
    g.TY = 64 - 2 * kHalo;
    g.tilesx = (p->nx + g.TX - 1) / g.TX;
  }
  return g;
}

int tiles(const pts_problem* p, const Geo& g) {
  if (g.whole) return 1;
  return g.tilesx * ((p->ny + g.TY - 1) / g.TY);
}

// Inner-solve plan: sweeps per pass and how passes are packed into launches.
struct Plan {
  int sweeps = 1;
  int passes = 1;          // total restarted passes per level
  std::vector<int> packs;  // passes per launch
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


// lvl_bits: 2 words per level (max |r|, max radius), zeroed here; scal (nullable)
// receives the maxima over levels.
int launch_residual(const pts_problem* p, const KProb& kp, const double* U, const double* u0, double* R,
                    double* coef, unsigned long long* lvl_bits, unsigned long long* scal, hipStream_t s) {
  const int tilesx = (p->nx + 63) / 64, tilesy = (p->ny + kResRows - 1) / kResRows;
  if (lvl_bits) hipLaunchKernelGGL(k_zero, dim3((2 * p->nt + 255) / 256), dim3(256), 0, s, lvl_bits, 2 * p->nt);
  dim3 grid((unsigned)(tilesx * tilesy), (unsigned)p->nt);
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, s, kp, U, u0, R, coef, lvl_bits);
  if (scal) hipLaunchKernelGGL(k_level_max, dim3(1), dim3(256), 0, s, lvl_bits, p->nt, scal);
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

// Forward block substitution over all levels: du^n = A_n^{-1}(r^n + du^{n-1}) (Eq. (7)).
struct Prof;
void prof_begin(Prof* pr, int kind, hipStream_t s);
void prof_end(Prof* pr, hipStream_t s, double bytes);

int launch_chain(const pts_problem* p, const KProb& kp, const double* U, const double* R, double* dU, double* Xs,
                 const double* rho, const Plan& pl, const Geo& g, hipStream_t s, int* launches, Prof* pr) {
  const size_t ns = (size_t)p->nx * p->ny;
  const int nb = tiles(p, g);
  const int nl = (int)pl.packs.size();
  for (int n = 0; n < p->nt; ++n) {
    const double* prev = n == 0 ? nullptr : dU + (size_t)(n - 1) * ns;
    double* out = dU + (size_t)n * ns;
    // ping-pong between the scratch level and dU[n] so that the last launch writes dU[n]
    const double* xin = nullptr;
    for (int l = 0; l < nl; ++l) {
      double* xo = ((nl - 1 - l) % 2 == 0) ? out : Xs;
      prof_begin(pr, 1, s);
      if (pl.fp32)
        hipLaunchKernelGGL(k_level_solve<float>, dim3(nb), dim3(512), 0, s, kp, n, U, R, prev, xin, xo, rho, g,
                           pl.packs[l], pl.sweeps);
      else
        hipLaunchKernelGGL(k_level_solve<double>, dim3(nb), dim3(512), 0, s, kp, n, U, R, prev, xin, xo, rho, g,
                           pl.packs[l], pl.sweeps);
      prof_end(pr, s, 8.0 * (double)ns * (3 + (prev ? 1 : 0) + (xin ? 1 : 0)));
      xin = xo;
      ++*launches;
    }
  }
  HIPCHK(hipGetLastError());
  return PTS_OK;
}

struct HostScalars {
  double* h = nullptr;  // pinned: [0] max|r|, [1] rho_max, [2] sum dU^2
  ~HostScalars() {
    if (h) (void)hipHostFree(h);
  }
};
thread_local HostScalars g_host;

int host_scalars(double** out) {
  if (!g_host.h) HIPCHK(hipHostMalloc((void**)&g_host.h, 64, hipHostMallocDefault));
  *out = g_host.h;
  return PTS_OK;
}

// Optional per-kernel timing with HIP events recorded on the launch stream.
struct Prof {
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  double bytes = 0.0;
  void begin(int kind, hipStream_t s) {
    Rec r{kind, nullptr, nullptr};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end(hipStream_t s) { (void)hipEventRecord(recs.back().b, s); }
  void collect(pts_stats* st) {
    for (auto& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && st) {
        st->prof_ms[r.kind] += ms;
        st->prof_count[r.kind] += 1;
      }
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    recs.clear();
    if (st) st->level_solve_bytes = bytes;
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
  int residual(const double* U, const double* u0, hipStream_t s, int* launches) {
    *launches += 3;
    prof_begin(prof, 0, s);
    int rc = launch_residual(p, kp, U, u0, R, nullptr, rho, scal, s);
    if (prof) prof->end(s);
    return rc;
  }

  int step_body(double* U, const Plan& pl, hipStream_t s, int* launches) {
    int rc = launch_chain(p, kp, U, R, dU, Xs, (const double*)rho, pl, g, s, launches, prof);
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
  if (o->window > 1) return fail(PTS_ERR_INVALID_ARG, "window %d: only window 1 is available", o->window);
  if (o->window < 0 || o->sweeps < 0 || o->lin_tol < 0)
    return fail(PTS_ERR_INVALID_ARG, "negative option");
  if (o->schedule != PTS_SCHED_AUTO && o->schedule != PTS_SCHED_BULK)
    return fail(PTS_ERR_INVALID_ARG, "schedule %d not available", o->schedule);
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

int solve_bulk(const pts_problem* p, double* U, const double* u0, double tol, int max_iter, void* ws,
               const pts_options* o, pts_stats* st, hipStream_t s, bool single_step) {
  Instance in;
  in.bind(p, ws);
  Prof prof;
  const bool profiling = o && o->profile;
  if (profiling) in.prof = &prof;
  double* hs;
  int rc = host_scalars(&hs);
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
    if (rhom >= 1.0) {
      if (st) st->iterations = it;
      return fail(PTS_ERR_SINGULAR, "block A_n not diagonally dominant (Gershgorin radius %.3g)", rhom);
    }
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
      st->sweeps = pl.sweeps;
      st->refine = pl.passes - 1;
      st->window = 1;
      st->schedule = PTS_SCHED_BULK;
    }
    if (use_graph) {
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

}  // namespace

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
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, s, kp, U, u0, R, coef, nullptr);
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
  return solve_bulk(p, U, u0, 0.0, 1, workspace, opts, stats, (hipStream_t)stream, true);
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
  rc = solve_bulk(p, U, u0, tol, max_iter, workspace, opts, stats, (hipStream_t)stream, false);
  if (stats)
    stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

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
  return t;
}

int pts_solve_batched(const pts_problem* probs, int nprob, double* const* U, const double* const* u0, double tol,
                      int max_iter, void* workspace, size_t workspace_bytes, const pts_options* opts,
                      pts_stats* stats, pts_stream_t stream) {
  const size_t need = pts_workspace_bytes_batched(probs, nprob);
  if (need == 0) return PTS_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < need) return fail(PTS_ERR_WORKSPACE, "batched workspace too small");
  char* w = (char*)workspace;
  int worst = PTS_OK;
  for (int i = 0; i < nprob; ++i) {
    const size_t b = layout(probs + i).total;
    int rc = pts_solve(probs + i, U[i], u0[i], tol, max_iter, w, b, opts, stats ? stats + i : nullptr, stream);
    if (rc && !worst) worst = rc;
    w += b;
  }
  return worst;
}

}  // extern "C"
