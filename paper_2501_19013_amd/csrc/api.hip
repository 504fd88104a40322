// C ABI entry points (include/fcw.h): argument checks, context lifetime, call order,
// buffer management and the step loop.  All numerical work runs in the kernels of
// setup.hip, step.hip and lanczos.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>

#include "common.h"

namespace fcw {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

fcw_status hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FCW_E_NOMEM : FCW_E_DEVICE;
}

template <typename P>
static fcw_status dmalloc(Ctx& c, P** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  c.footprint += (int64_t)bytes;
  return FCW_OK;
}

template <typename P>
static void dfree(P*& ptr) {
  if (ptr) (void)hipFree((void*)ptr);
  ptr = nullptr;
}

static void free_all(Ctx& c) {
  dfree(c.d_void_c); dfree(c.d_void_r); dfree(c.d_cls); dfree(c.d_info);
  dfree(c.d_cut_cells); dfree(c.d_cut_vptr); dfree(c.d_cut_vidx); dfree(c.d_all_void);
  dfree(c.d_tab); dfree(c.d_kref); dfree(c.d_mfull); dfree(c.d_lref); dfree(c.d_kcut);
  dfree(c.d_mcut); dfree(c.d_lumped); dfree(c.d_margin); dfree(c.d_evs_fail); dfree(c.d_mass);
  dfree(c.d_invm); dfree(c.d_kref_s); dfree(c.d_kcut_s); dfree(c.d_invm64); dfree(c.d_ubuf); dfree(c.d_ycut);
  dfree(c.d_invw); dfree(c.d_mflag); dfree(c.d_kref_bf);
  dfree(c.d_src);
  dfree(c.d_goff);
  dfree(c.d_gdof);
  dfree(c.d_gval);
  dfree(c.d_rec);
  dfree(c.d_red);
  if (c.h_red) (void)hipHostFree(c.h_red);
  c.h_red = nullptr;
  imex_free(c);
  dfree(c.d_wl);
  if (c.h_wl) (void)hipHostFree(c.h_wl);
  c.h_wl = nullptr;
  if (c.wl_event) (void)hipEventDestroy(c.wl_event);
  c.wl_event = nullptr;
  if (c.graph_exec) (void)hipGraphExecDestroy(c.graph_exec);
  c.graph_exec = nullptr;
}

static bool in_any_void(const Ctx& c, const double* x) {
  if (c.cube.on && cube_point_outside(c.cube, x)) return true;
  for (int v = 0; v < c.nvoids; ++v) {
    double d2 = 0.0;
    for (int k = 0; k < c.dim; ++k) {
      const double t = x[k] - c.void_c[(size_t)v * c.dim + k];
      d2 += t * t;
    }
    if (d2 < c.void_r[v] * c.void_r[v]) return true;
  }
  return false;
}

static fcw_status check_ctx(const fcw_ctx* ctx, int need_state) {
  if (!ctx) {
    set_error("null context");
    return FCW_E_ARG;
  }
  if (ctx->poisoned) {
    set_error("context is unusable after a device error");
    return FCW_E_DEVICE;
  }
  if (ctx->state < need_state) {
    set_error("call out of order (context state %d, need %d)", ctx->state, need_state);
    return FCW_E_STATE;
  }
  return FCW_OK;
}

// Capture the launches `queue` makes on the context's stream into a graph and time one
// replay of it between events e0 and e1, so host-side gaps between short launches stay
// out of the figure.  An untimed replay goes first.  Synchronises.
template <typename F>
static fcw_status time_captured(Ctx& c, hipEvent_t e0, hipEvent_t e1, F queue) {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  hipError_t e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const fcw_status st = queue();
  e = hipStreamEndCapture(c.stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  e = hipGraphLaunch(x, c.stream);
  if (e == hipSuccess) e = hipEventRecord(e0, c.stream);
  if (e == hipSuccess) e = hipGraphLaunch(x, c.stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c.stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  (void)hipStreamSynchronize(c.stream);
  (void)hipGraphExecDestroy(x);
  return e == hipSuccess ? FCW_OK : hip_fail(e, "kernel timing replay");
}

// checks of one problem's step call
fcw_status check_step_call(const fcw_ctx* c, int32_t nrhs, const void* u, const void* d,
                           const fcw_source* src, double dt, int32_t nsteps) {
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (nrhs < 1 || nrhs > 64 || !u || !d || !(dt > 0.0) || nsteps < 0) {
    set_error("invalid arguments (nrhs in [1,64], u, d non-null, dt > 0, nsteps >= 0)");
    return FCW_E_ARG;
  }
  if (src) {
    for (int s = 0; s < nrhs; ++s) {
      for (int k = 0; k < c->dim; ++k)
        if (!(src[s].x[k] >= c->lo[k] && src[s].x[k] <= c->hi[k])) {
          set_error("source %d outside the box", s);
          return FCW_E_ARG;
        }
      if (in_any_void(*c, src[s].x)) {
        set_error("source %d lies inside a void", s);
        return FCW_E_ARG;
      }
      if (!(src[s].f0 > 0.0)) {
        set_error("source %d needs f0 > 0", s);
        return FCW_E_ARG;
      }
    }
  }
  return FCW_OK;
}

// The work queued after each step of a call by fcw_run / fcw_step_explicit: volumetric
// loads of the next step, then receiver samples of the state just written.
struct StepObservers {
  std::vector<LoadTarget> loads;
  std::vector<TraceTarget> traces;
  bool empty() const { return loads.empty() && traces.empty(); }
  static fcw_status fn(void* arg, hipStream_t s, int j) {
    StepObservers* o = static_cast<StepObservers*>(arg);
    fcw_status st = launch_gauss_loads(s, o->loads.data(), (int)o->loads.size(), j);
    if (st) return st;
    return launch_traces(s, o->traces.data(), (int)o->traces.size(), j);
  }
};

void clear_error() { g_err.clear(); }

static fcw_status refuse_volumetric(const fcw_source* src, int nrhs) {
  if (src)
    for (int r = 0; r < nrhs && r < kMaxSrc; ++r)
      if (src[r].sigma > 0.0) {
        set_error("volumetric sources are taken by fcw_step_explicit and fcw_run only");
        return FCW_E_UNSUPPORTED;
      }
  return FCW_OK;
}

}  // namespace fcw

using namespace fcw;

extern "C" {

const char* fcw_last_error(void) { return g_err.c_str(); }

fcw_status fcw_assemble_cells(const fcw_problem_desc* desc, fcw_ctx** out) {
  g_err.clear();
  if (!desc || !out) {
    set_error("null argument");
    return FCW_E_ARG;
  }
  *out = nullptr;
  const fcw_problem_desc& d = *desc;
  if (d.dim != 2 && d.dim != 3) { set_error("dim must be 2 or 3"); return FCW_E_ARG; }
  if (!(d.ncomp == 1 || (d.ncomp == 3 && d.dim == 3))) {
    set_error("ncomp must be 1, or 3 with dim 3");
    return FCW_E_ARG;
  }
  if (d.p < 1 || d.p > kMaxP) { set_error("p must be in [1, %d]", kMaxP); return FCW_E_ARG; }
  if (d.tree_depth < 0 || d.dim * d.tree_depth > 10) {
    set_error("tree_depth must satisfy 0 <= dim*depth <= 10 (got %d)", d.tree_depth);
    return FCW_E_ARG;
  }
  if (d.nvoids < 0 || (d.nvoids > 0 && (!d.void_center || !d.void_radius))) {
    set_error("invalid void arrays");
    return FCW_E_ARG;
  }
  if (!(d.alpha >= 0.0) || !(d.rho > 0.0)) { set_error("need alpha >= 0, rho > 0"); return FCW_E_ARG; }
  if (!(d.cube_half >= 0.0)) { set_error("need cube_half >= 0"); return FCW_E_ARG; }
  if (d.ncomp == 1 && !(d.c > 0.0)) { set_error("need c > 0"); return FCW_E_ARG; }
  if (d.ncomp == 3 && !(d.E > 0.0 && d.nu > -1.0 && d.nu < 0.5)) {
    set_error("need E > 0 and -1 < nu < 0.5");
    return FCW_E_ARG;
  }
  if (d.precision != FCW_FP64 && d.precision != FCW_FP32 && d.precision != FCW_BF16) {
    set_error("precision %d not built", d.precision);
    return FCW_E_UNSUPPORTED;
  }
  double h = 0.0;
  for (int k = 0; k < d.dim; ++k) {
    if (d.ncells[k] < 1 || !(d.hi[k] > d.lo[k])) { set_error("empty grid"); return FCW_E_ARG; }
    const double hk = (d.hi[k] - d.lo[k]) / d.ncells[k];
    if (k == 0) h = hk;
    else if (std::fabs(hk - h) > 1e-14 * h) { set_error("cells must be cubes"); return FCW_E_ARG; }
  }
  fcw_ctx* c = new (std::nothrow) fcw_ctx();
  if (!c) { set_error("host allocation failed"); return FCW_E_NOMEM; }
  c->dim = d.dim;
  c->ncomp = d.ncomp;
  c->p = d.p;
  c->depth = d.tree_depth;
  c->precision = d.precision;
  c->h = h;
  c->alpha = d.alpha;
  c->rho = d.rho;
  c->c = d.c;
  c->E = d.E;
  c->nu = d.nu;
  c->stream = (hipStream_t)d.stream;
  c->ncell_total = 1;
  c->nnodes = 1;
  for (int k = 0; k < 3; ++k) {
    c->ncells[k] = (k < d.dim) ? d.ncells[k] : 1;
    c->npts[k] = (k < d.dim) ? d.ncells[k] * d.p + 1 : 1;
    c->lo[k] = (k < d.dim) ? d.lo[k] : 0.0;
    c->hi[k] = (k < d.dim) ? d.hi[k] : 0.0;
    c->ncell_total *= c->ncells[k];
    c->nnodes *= c->npts[k];
  }
  c->ndof = c->nnodes * c->ncomp;
  c->n_s = ipow(d.p + 1, d.dim);
  c->n_loc = c->n_s * d.ncomp;
  c->nvoids = d.nvoids;
  c->void_c.assign(d.void_center, d.void_center + (size_t)d.nvoids * d.dim);
  c->void_r.assign(d.void_radius, d.void_radius + d.nvoids);
  if (d.cube_half > 0.0) {
    c->cube.on = 1;
    c->cube.dim = d.dim;
    c->cube.a = d.cube_half;
    for (int k = 0; k < 3; ++k) c->cube.c[k] = (k < d.dim) ? d.cube_center[k] : 0.0;
    for (int k = 0; k < 9; ++k) c->cube.T[k] = d.cube_rot[k];
  }
  if (!step_supported(*c)) {
    set_error("no step kernel built for dim=%d p=%d ncomp=%d", d.dim, d.p, d.ncomp);
    delete c;
    return FCW_E_UNSUPPORTED;
  }

  auto fail = [&](fcw_status st) {
    free_all(*c);
    delete c;
    return st;
  };
  fcw_status st;
  const size_t nl2 = (size_t)c->n_loc * c->n_loc, ns2 = (size_t)c->n_s * c->n_s;
  if ((st = dmalloc(*c, &c->d_void_c, (size_t)d.nvoids * d.dim * 8)) ||
      (st = dmalloc(*c, &c->d_void_r, (size_t)d.nvoids * 8)) ||
      (st = dmalloc(*c, &c->d_cls, (size_t)c->ncell_total)) ||
      (st = dmalloc(*c, &c->d_info, (size_t)c->ncell_total * 4)) ||
      (st = dmalloc(*c, &c->d_tab, sizeof(RefTables))) ||
      (st = dmalloc(*c, &c->d_kref, nl2 * 8)) || (st = dmalloc(*c, &c->d_mfull, ns2 * 8)) ||
      (st = dmalloc(*c, &c->d_lref, (size_t)c->n_s * 8)))
    return fail(st);
  if (d.nvoids > 0) {
    if (hipMemcpyAsync(c->d_void_c, d.void_center, (size_t)d.nvoids * d.dim * 8,
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_void_r, d.void_radius, (size_t)d.nvoids * 8, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
      return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync"));
  }
  if ((st = setup_reference(*c)) || (st = setup_classify(*c))) return fail(st);
  const size_t nc = (size_t)(c->n_cut_cand > 0 ? c->n_cut_cand : 1);
  if ((st = dmalloc(*c, &c->d_kcut, nc * nl2 * 8)) || (st = dmalloc(*c, &c->d_mcut, nc * ns2 * 8)) ||
      (st = dmalloc(*c, &c->d_lumped, nc * c->n_s * 8)) ||
      (st = dmalloc(*c, &c->d_margin, nc * 8)))
    return fail(st);
  if ((st = setup_integrate(*c))) return fail(st);
  if ((st = setup_reclassify(*c))) return fail(st);
  c->state = 1;
  *out = c;
  return FCW_OK;
}

fcw_status fcw_stabilize_cut_cells(fcw_ctx* c, double eps, double f_lambda) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  if (!(eps >= 0.0) || !(f_lambda > 0.0 && f_lambda < 1.0)) {
    set_error("need eps >= 0 and 0 < f_lambda < 1");
    return FCW_E_ARG;
  }
  const size_t sb = c->state_bytes();
  const size_t nl = c->n_loc;
  const size_t npk = nl * (nl + 1) / 2;
  const size_t nc = (size_t)(c->n_cut_cand > 0 ? c->n_cut_cand : 1);
  if (!c->d_mass) {
    if ((st = dmalloc(*c, &c->d_mass, c->nnodes * 8)) ||
        (st = dmalloc(*c, &c->d_invm64, c->nnodes * 8)) ||
        (st = dmalloc(*c, &c->d_invm, c->nnodes * sb)) ||
        (st = dmalloc(*c, &c->d_kref_s, nl * nl * sb)) ||
        (st = dmalloc(*c, &c->d_kcut_s, nc * npk * sb)))
      return st;
  }
  if ((st = setup_stabilize(*c, eps, f_lambda))) return st;
  if ((st = setup_mass_and_pack(*c))) return st;
  // smallest classification margin of the eigenvalue split over the kept cut cells
  c->min_margin = 0.0;
  if (c->n_cut_cand > 0 && eps != 0.0) {
    std::vector<double> m(c->n_cut_cand);
    std::vector<int32_t> av(c->n_cut_cand);
    FCW_HIP(hipMemcpyAsync(m.data(), c->d_margin, m.size() * 8, hipMemcpyDeviceToHost, c->stream));
    FCW_HIP(hipMemcpyAsync(av.data(), c->d_all_void, av.size() * 4, hipMemcpyDeviceToHost,
                           c->stream));
    FCW_HIP(hipStreamSynchronize(c->stream));
    double mm = 1e300;
    for (size_t i = 0; i < m.size(); ++i)
      if (!av[i]) mm = std::fmin(mm, m[i]);
    c->min_margin = mm;
  }
  c->state = 2;
  c->dt_crit = 0.0;
  return FCW_OK;
}

fcw_status fcw_critical_dt(fcw_ctx* c, int32_t max_iter, double rtol, double* dt_crit) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (!dt_crit || max_iter < 2 || !(rtol > 0.0)) {
    set_error("need dt_crit != NULL, max_iter >= 2, rtol > 0");
    return FCW_E_ARG;
  }
  double lmax = 0.0;
  if ((st = lanczos_lambda_max(*c, max_iter, rtol, &lmax))) return st;
  c->dt_crit = 2.0 / std::sqrt(lmax);
  *dt_crit = c->dt_crit;
  return FCW_OK;
}

// checks of one problem's step call; prepares its sources and scratch
static fcw_status prepare_call(fcw_ctx* c, int32_t nrhs, void* u, void* d, const fcw_source* src,
                               double dt, int32_t nsteps) {
  fcw_status st = check_step_call(c, nrhs, u, d, src, dt, nsteps);
  if (st) return st;
  if (src && (st = prepare_sources(*c, nrhs, src))) return st;
  const size_t bytes = (size_t)nrhs * c->ndof * c->state_bytes();
  if (c->ubuf_bytes < bytes) {
    dfree(c->d_ubuf);
    c->footprint -= (int64_t)c->ubuf_bytes;
    c->ubuf_bytes = 0;
    if ((st = dmalloc(*c, &c->d_ubuf, bytes))) return st;
    c->ubuf_bytes = bytes;
  }
  return FCW_OK;
}

fcw_status fcw_run(const fcw_run_item* items, int32_t n, int32_t flags) {
  g_err.clear();
  if (!items || n < 1) {
    set_error("need at least one run item");
    return FCW_E_ARG;
  }
  fcw_ctx* owner = items[0].ctx;
  fcw_status st = check_ctx(owner, 2);
  if (st) return st;
  // validate and prepare every member first (no step is enqueued on error)
  std::vector<double> dts(n);
  int check_every = 0;
  bool any_rec = false, sync_end = false;
  for (int i = 0; i < n; ++i) {
    const fcw_run_item& r = items[i];
    if (!r.ctx) { set_error("run item %d has no context", i); return FCW_E_ARG; }
    double dt = r.dt;
    if (!(dt > 0.0)) {
      // step size rule of Sec. 3.3: dt = min(0.9 dt_crit, dt_max)
      if (!(r.ctx->dt_crit > 0.0)) {
        set_error("run item %d: dt <= 0 needs fcw_critical_dt first", i);
        return FCW_E_STATE;
      }
      dt = 0.9 * r.ctx->dt_crit;
      if (r.dt_max > 0.0 && r.dt_max < dt) dt = r.dt_max;
    }
    dts[i] = dt;
    for (int k = 0; k < i; ++k)
      if (items[k].ctx == r.ctx) { set_error("context listed twice in one run"); return FCW_E_ARG; }
    if (r.nrec < 0 || r.nrec > FCW_MAX_RECEIVERS || (r.nrec > 0 && (!r.rec_x || !r.traces))) {
      set_error("run item %d: need 0 <= nrec <= %d, and points and a trace buffer with nrec > 0",
                i, FCW_MAX_RECEIVERS);
      return FCW_E_ARG;
    }
    for (int q = 0; q < r.nrec; ++q) {
      const double* x = r.rec_x + 3 * q;
      for (int k = 0; k < r.ctx->dim; ++k)
        if (!(x[k] >= r.ctx->lo[k] && x[k] <= r.ctx->hi[k])) {
          set_error("run item %d: receiver %d outside the box", i, q);
          return FCW_E_ARG;
        }
    }
    if (r.check_every < 0 || (r.check_every > 0 && check_every > 0 && r.check_every != check_every)) {
      set_error("run item %d: check_every must be >= 0 and the same for every item that checks", i);
      return FCW_E_ARG;
    }
    if (r.check_every > 0) check_every = r.check_every;
    any_rec = any_rec || r.nrec > 0;
    sync_end = sync_end || r.result || r.energy || r.check_every > 0;
    if ((st = check_step_call(r.ctx, r.nrhs, r.u, r.d, r.src, dt, r.nsteps))) return st;
  }
  for (int i = 0; i < n; ++i) {
    const fcw_run_item& r = items[i];
    if ((st = prepare_call(r.ctx, r.nrhs, r.u, r.d, r.src, dts[i], r.nsteps))) return st;
    r.ctx->d_src_active = r.src != nullptr;
    if (r.nrec > 0 && (st = prepare_receivers(*r.ctx, r.nrec, r.rec_x))) return st;
  }
  // per item: steps done, outcome, growth-check history per right-hand side
  struct ItemRun {
    int done = 0;
    fcw_status status = FCW_OK;
    double growth = 0.0;
    std::vector<double> prev;
    std::vector<int> streak;
  };
  std::vector<ItemRun> ir(n);
  int maxsteps = 0;
  for (int i = 0; i < n; ++i) {
    ir[i].prev.assign(items[i].nrhs, 0.0);
    ir[i].streak.assign(items[i].nrhs, 0);
    maxsteps = std::max(maxsteps, items[i].nsteps);
  }
  const int chunk = check_every > 0 ? check_every : std::max(maxsteps, 1);
  const bool graph = (flags & FCW_RUN_GRAPH) != 0 && !any_rec;
  bool any_load = false;
  for (int i = 0; i < n; ++i) any_load = any_load || (items[i].src && items[i].ctx->g_active);
  const bool graph2 = graph && !any_load;
  for (;;) {
    // the next chunk of steps of every problem still running
    std::vector<GroupMember> group;
    std::vector<int> solo, cnt(n, 0);
    StepObservers ghook;
    bool more = false;
    for (int i = 0; i < n; ++i) {
      const fcw_run_item& r = items[i];
      if (ir[i].status != FCW_OK) continue;
      const int k = std::min(chunk, r.nsteps - ir[i].done);
      if (k <= 0) continue;
      more = true;
      cnt[i] = k;
      const double t0 = r.t0 + ir[i].done * dts[i];
      const int start = (r.start && ir[i].done == 0) ? 1 : 0;
      if (groupable_2d(*owner, *r.ctx) || groupable_3d(*owner, *r.ctx)) {
        group.push_back(GroupMember{r.ctx, r.nrhs, r.u, r.d, r.ctx->d_ubuf, t0, dts[i], k, start});
        if (r.nrec > 0)
          ghook.traces.push_back(TraceTarget{r.ctx, r.u, r.ctx->d_ubuf, r.nrhs, k, r.nrec,
                                             r.traces, (int64_t)r.nsteps + 1,
                                             (int64_t)ir[i].done});
        if (r.src && r.ctx->g_active)
          ghook.loads.push_back(LoadTarget{r.ctx, r.d, r.nrhs, k, start, t0, dts[i]});
      } else {
        solo.push_back(i);
      }
    }
    if (!more) break;
    // the group runs on the owner's stream; sources of members without any are hidden
    std::vector<SourceDev*> saved;
    for (auto& g : group) {
      saved.push_back(g.ctx->d_src);
      if (!g.ctx->d_src_active) g.ctx->d_src = nullptr;
    }
    const StepHook gh{StepObservers::fn, &ghook};
    if (!group.empty())
      st = (owner->dim == 3)
               ? run_group3d(*owner, group, graph2, ghook.empty() ? nullptr : &gh)
               : run_group(*owner, group, graph2, ghook.empty() ? nullptr : &gh);
    for (size_t k = 0; k < group.size(); ++k) group[k].ctx->d_src = saved[k];
    if (st) return st;
    for (int i : solo) {
      const fcw_run_item& r = items[i];
      fcw_ctx* c = r.ctx;
      StepObservers sh;
      const int sstart = (r.start && ir[i].done == 0) ? 1 : 0;
      if (r.nrec > 0)
        sh.traces.push_back(TraceTarget{c, r.u, c->d_ubuf, r.nrhs, cnt[i], r.nrec, r.traces,
                                        (int64_t)r.nsteps + 1, (int64_t)ir[i].done});
      if (r.src && c->g_active)
        sh.loads.push_back(
            LoadTarget{c, r.d, r.nrhs, cnt[i], sstart, r.t0 + ir[i].done * dts[i], dts[i]});
      const StepHook hk{StepObservers::fn, &sh};
      SourceDev* sv = c->d_src;
      if (!r.src) c->d_src = nullptr;
      hipStream_t s0 = c->stream;
      c->stream = owner->stream;
      st = run_steps(*c, c->tile_choice, r.nrhs, r.u, r.d, c->d_ubuf,
                     r.t0 + ir[i].done * dts[i], dts[i], cnt[i], sstart,
                     sh.empty() ? nullptr : &hk);
      c->stream = s0;
      c->d_src = sv;
      if (st) return st;
    }
    for (int i = 0; i < n; ++i) ir[i].done += cnt[i];
    if (check_every == 0) continue;
    // growth checks (Sec. 2.3): sum d_i^2 per right-hand side after the chunk
    for (int i = 0; i < n; ++i) {
      const fcw_run_item& r = items[i];
      if (r.check_every == 0 || cnt[i] == 0) continue;
      if ((st = state_sums(*r.ctx, owner->stream, r.nrhs, nullptr, r.d, nullptr, false)))
        return st;
      ItemRun& x = ir[i];
      double g = 0.0;
      for (int q = 0; q < r.nrhs; ++q) {
        const double sq = r.ctx->h_red[3 * q];
        if (!std::isfinite(sq)) {
          x.status = FCW_E_UNSTABLE;
          g = sq;
          break;
        }
        if (x.prev[q] > 0.0) {
          const double ratio = sq / x.prev[q];
          g = std::max(g, ratio);
          x.streak[q] = ratio > 1e6 ? x.streak[q] + 1 : 0;
          if (x.streak[q] >= 3) x.status = FCW_E_UNSTABLE;
        }
        x.prev[q] = sq;
      }
      x.growth = g;
    }
  }
  // energies after the last step: r = K u in the partner buffer, then the three sums
  for (int i = 0; i < n; ++i) {
    const fcw_run_item& r = items[i];
    if (!r.energy) continue;
    fcw_ctx* c = r.ctx;
    hipStream_t s0 = c->stream;
    c->stream = owner->stream;
    st = launch_apply(*c, r.nrhs, r.u, c->d_ubuf);
    c->stream = s0;
    if (st) return st;
    if ((st = state_sums(*c, owner->stream, r.nrhs, r.u, r.d, c->d_ubuf, true))) return st;
    const double dt = dts[i];
    for (int q = 0; q < r.nrhs; ++q) {
      const double* t = c->h_red + 3 * q;
      r.energy[q] = 0.5 * (t[0] / (dt * dt) + t[1] - t[2]);
    }
  }
  if (sync_end) FCW_HIP(hipStreamSynchronize(owner->stream));
  bool unstable = false;
  for (int i = 0; i < n; ++i) {
    if (items[i].result) {
      items[i].result->status = ir[i].status;
      items[i].result->steps_done = ir[i].done;
      items[i].result->dt_used = dts[i];
      items[i].result->growth = ir[i].growth;
    }
    unstable = unstable || ir[i].status == FCW_E_UNSTABLE;
  }
  if (unstable) {
    std::string which;
    for (int i = 0; i < n; ++i)
      if (ir[i].status == FCW_E_UNSTABLE) which += " " + std::to_string(i);
    set_error("growth detected (dt above the critical step?) in run item(s)%s", which.c_str());
    return FCW_E_UNSTABLE;
  }
  return FCW_OK;
}

fcw_status fcw_step_explicit(fcw_ctx* c, int32_t nrhs, void* u, void* d, const fcw_source* src,
                             double t0, double dt, int32_t nsteps, int32_t start) {
  g_err.clear();
  fcw_status st = prepare_call(c, nrhs, u, d, src, dt, nsteps);
  if (st) return st;
  if (nsteps == 0) return FCW_OK;
  SourceDev* saved = c->d_src;
  if (!src) c->d_src = nullptr;
  StepObservers ob;
  if (src && c->g_active) ob.loads.push_back(LoadTarget{c, d, nrhs, nsteps, start, t0, dt});
  const StepHook hk{StepObservers::fn, &ob};
  st = run_steps(*c, c->tile_choice, nrhs, u, d, c->d_ubuf, t0, dt, nsteps, start,
                 ob.empty() ? nullptr : &hk);
  c->d_src = saved;
  return st;
}

fcw_status fcw_autotune(fcw_ctx* c, int32_t nrhs, int32_t nsteps, int32_t* chosen) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (nrhs < 1 || nrhs > 64 || nsteps < 1) {
    set_error("need 1 <= nrhs <= 64 and nsteps >= 1");
    return FCW_E_ARG;
  }
  const int n = tile_candidates(*c, -1, nullptr);
  const size_t bytes = (size_t)nrhs * c->ndof * c->state_bytes();
  void *ua = nullptr, *ub = nullptr, *dd = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (ua) (void)hipFree(ua);
    if (ub) (void)hipFree(ub);
    if (dd) (void)hipFree(dd);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&ua, bytes) != hipSuccess || hipMalloc(&ub, bytes) != hipSuccess ||
      hipMalloc(&dd, bytes) != hipSuccess) {
    cleanup();
    set_error("autotune scratch allocation failed");
    return FCW_E_NOMEM;
  }
  if (hipMemsetAsync(ua, 0, bytes, c->stream) != hipSuccess ||
      hipMemsetAsync(dd, 0, bytes, c->stream) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return hip_fail(hipGetLastError(), "autotune setup");
  }
  const SourceDev* saved = c->d_src;
  c->d_src = nullptr;
  c->tune_us.assign(n, 0.0);
  int best = 0;
  void* sc = nullptr;
  if (hipMalloc(&sc, bytes) != hipSuccess) {
    cleanup();
    set_error("autotune scratch allocation failed");
    return FCW_E_NOMEM;
  }
  for (int i = 0; i < n && st == FCW_OK; ++i) {
    st = run_steps(*c, i, nrhs, ua, dd, sc, 0.0, 1e-6, 2, 0);  // warm-up
    if (st) break;
    (void)hipEventRecord(e0, c->stream);
    st = run_steps(*c, i, nrhs, ua, dd, sc, 0.0, 1e-6, nsteps, 0);
    (void)hipEventRecord(e1, c->stream);
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = hip_fail(hipGetLastError(), "autotune timing");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    c->tune_us[i] = 1000.0 * ms / nsteps;
    if (c->tune_us[i] < c->tune_us[best]) best = i;
  }
  (void)hipFree(sc);
  c->d_src = const_cast<SourceDev*>(saved);
  cleanup();
  if (st) return st;
  c->tile_choice = best;
  if (chosen) *chosen = best;
  return FCW_OK;
}

fcw_status fcw_tile_config(const fcw_ctx* c, int32_t i, int32_t tile[3], double* us_per_step,
                           int32_t* count) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  int t[3] = {0, 0, 0};
  const int n = tile_candidates(*c, i, t);
  if (count) *count = n;
  if (i < 0 || i >= n) {
    set_error("tile configuration %d out of range [0, %d)", i, n);
    return FCW_E_ARG;
  }
  if (tile)
    for (int k = 0; k < 3; ++k) tile[k] = t[k];
  if (us_per_step) *us_per_step = (i < (int)c->tune_us.size()) ? c->tune_us[i] : 0.0;
  return FCW_OK;
}

fcw_status fcw_tile_name(const fcw_ctx* c, int32_t i, char* buf, int32_t cap) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  std::string name;
  const int n = tile_candidates(*c, i, nullptr, &name);
  if (i < 0 || i >= n) {
    set_error("tile configuration %d out of range [0, %d)", i, n);
    return FCW_E_ARG;
  }
  if (!buf || cap < (int32_t)name.size() + 1) {
    set_error("name buffer needs %d bytes", (int)name.size() + 1);
    return FCW_E_ARG;
  }
  std::memcpy(buf, name.c_str(), name.size() + 1);
  return FCW_OK;
}

fcw_status fcw_select_tile(fcw_ctx* c, int32_t i) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  const int n = tile_candidates(*c, -1, nullptr);
  if (i < 0 || i >= n) {
    set_error("tile configuration %d out of range [0, %d)", i, n);
    return FCW_E_ARG;
  }
  c->tile_choice = i;
  return FCW_OK;
}

fcw_status fcw_set_stream(fcw_ctx* c, void* stream) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  // work already queued on the old stream completes before later work is queued elsewhere
  FCW_HIP(hipStreamSynchronize(c->stream));
  c->stream = (hipStream_t)stream;
  return FCW_OK;
}

fcw_status fcw_kernel_times(fcw_ctx* c, int32_t nrhs, int32_t nsteps, double* main_us,
                            double* cut_us) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (nrhs < 1 || nrhs > 64 || nsteps < 1 || !main_us || !cut_us) {
    set_error("need 1 <= nrhs <= 64, nsteps >= 1 and non-null outputs");
    return FCW_E_ARG;
  }
  const size_t bytes = (size_t)nrhs * c->ndof * c->state_bytes();
  // the work goes on a private stream (the default stream cannot be captured) after
  // everything queued on the context's stream
  FCW_HIP(hipStreamSynchronize(c->stream));
  hipStream_t own = nullptr;
  FCW_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  c->stream = own;
  void *ua = nullptr, *dd = nullptr, *sc = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(own);
    c->stream = user;
    (void)hipStreamDestroy(own);
    if (ua) (void)hipFree(ua);
    if (dd) (void)hipFree(dd);
    if (sc) (void)hipFree(sc);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (hipMalloc(&ua, bytes) != hipSuccess || hipMalloc(&dd, bytes) != hipSuccess ||
      hipMalloc(&sc, bytes) != hipSuccess) {
    cleanup();
    set_error("kernel timing scratch allocation failed");
    return FCW_E_NOMEM;
  }
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      cleanup();
      return hip_fail(hipGetLastError(), "kernel timing events");
    }
  if (hipMemsetAsync(ua, 0, bytes, c->stream) != hipSuccess ||
      hipMemsetAsync(dd, 0, bytes, c->stream) != hipSuccess) {
    cleanup();
    return hip_fail(hipGetLastError(), "kernel timing setup");
  }
  const SourceDev* saved = c->d_src;
  c->d_src = nullptr;
  // the cut-cell kernel back to back, then the main kernel back to back on its products;
  // a warm-up pass first, so buffers and kernel attributes are set before the capture
  if (!(st = run_steps(*c, c->tile_choice, nrhs, ua, dd, sc, 0.0, 1e-6, 2, 1)) &&
      c->n_cut_cand > 0)
    st = time_captured(*c, ev[0], ev[1], [&]() {
      fcw_status s2 = FCW_OK;
      for (int k = 0; k < nsteps && !s2; ++k) s2 = launch_cut_products(*c, nrhs, ua);
      return s2;
    });
  if (!st) {
    c->skip_cut = true;
    st = time_captured(*c, ev[2], ev[3], [&]() {
      return run_steps(*c, c->tile_choice, nrhs, ua, dd, sc, 0.0, 1e-6, nsteps, 0);
    });
    c->skip_cut = false;
  }
  c->d_src = const_cast<SourceDev*>(saved);
  if (!st) {
    float t0 = 0.0f, t1 = 0.0f;
    if ((c->n_cut_cand > 0 && hipEventElapsedTime(&t0, ev[0], ev[1]) != hipSuccess) ||
        hipEventElapsedTime(&t1, ev[2], ev[3]) != hipSuccess)
      st = hip_fail(hipGetLastError(), "kernel timing");
    *cut_us = c->n_cut_cand > 0 ? 1e3 * t0 / nsteps : 0.0;
    *main_us = 1e3 * t1 / nsteps;
  }
  cleanup();
  return st;
}

fcw_status fcw_imex_prepare(fcw_ctx* c, double dt, int64_t* n_c) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (c->precision != FCW_FP64) {
    set_error("the IMEX scheme runs on FP64 contexts only");
    return FCW_E_UNSUPPORTED;
  }
  if (!(dt > 0.0) || !n_c) {
    set_error("need dt > 0 and non-null n_c");
    return FCW_E_ARG;
  }
  if ((st = imex_prepare(*c, dt))) return st;
  *n_c = c->imex_nc;
  return FCW_OK;
}

fcw_status fcw_imex_layout(fcw_ctx* c, int32_t* n_blocks, int64_t* largest,
                           int64_t* solve_bytes) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (c->imex_nc < 0) {
    set_error("fcw_imex_prepare has not run");
    return FCW_E_ARG;
  }
  if (n_blocks) *n_blocks = c->imex_nblk;
  if (largest) *largest = c->imex_largest;
  if (solve_bytes) *solve_bytes = c->imex_ntiles * 32 * 32 * (int64_t)sizeof(double);
  return FCW_OK;
}

fcw_status fcw_step_imex(fcw_ctx* c, int32_t nrhs, void* u, void* d, void* v_c, void* a_c,
                         const fcw_source* src, double t0, double dt, int32_t nsteps,
                         int32_t start) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (c->precision != FCW_FP64) {
    set_error("the IMEX scheme runs on FP64 contexts only");
    return FCW_E_UNSUPPORTED;
  }
  if ((st = refuse_volumetric(src, nrhs))) return st;
  if ((st = prepare_call(c, nrhs, u, d, src, dt, nsteps))) return st;
  if ((st = imex_prepare(*c, dt))) return st;
  if (c->imex_nc > 0 && (!v_c || !a_c)) {
    set_error("v_c and a_c are needed (%lld implicit DOFs)", (long long)c->imex_nc);
    return FCW_E_ARG;
  }
  if (nsteps == 0) return FCW_OK;
  SourceDev* saved = c->d_src;
  if (!src) c->d_src = nullptr;
  st = imex_run(*c, nrhs, (double*)u, (double*)d, (double*)v_c, (double*)a_c, t0, dt, nsteps,
                start, false);
  c->d_src = saved;
  return st;
}

fcw_status fcw_step_consistent(fcw_ctx* c, int32_t nrhs, void* u, void* d, const fcw_source* src,
                               double t0, double dt, int32_t nsteps, int32_t start) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (c->precision != FCW_FP64) {
    set_error("the consistent-mass step runs on FP64 contexts only");
    return FCW_E_UNSUPPORTED;
  }
  if ((st = refuse_volumetric(src, nrhs))) return st;
  if ((st = prepare_call(c, nrhs, u, d, src, dt, nsteps))) return st;
  if ((st = imex_prepare(*c, dt))) return st;
  if (nsteps == 0) return FCW_OK;
  SourceDev* saved = c->d_src;
  if (!src) c->d_src = nullptr;
  st = imex_run(*c, nrhs, (double*)u, (double*)d, nullptr, nullptr, t0, dt, nsteps, start, true);
  c->d_src = saved;
  return st;
}

fcw_status fcw_apply_stiffness(fcw_ctx* c, int32_t nrhs, const void* u, void* r) {
  g_err.clear();
  fcw_status st = check_ctx(c, 2);
  if (st) return st;
  if (nrhs < 1 || nrhs > 65535 || !u || !r) {
    set_error("invalid arguments");
    return FCW_E_ARG;
  }
  return launch_apply(*c, nrhs, u, r);
}

fcw_status fcw_trace_error(const double* sim, int64_t sim_stride, const double* ref,
                           int64_t ref_stride, int32_t n_samples, int32_t n_obs, double* e) {
  g_err.clear();
  if (!sim || !ref || !e || sim_stride < 1 || ref_stride < 1 || n_samples < 1 || n_obs < 1) {
    set_error("need traces, strides >= 1, n_samples >= 1, n_obs >= 1 and an output");
    return FCW_E_ARG;
  }
  double sum = 0.0;
  for (int i = 0; i < n_obs; ++i) {
    double num = 0.0, den = 0.0;
    for (int64_t s = 1; s <= n_samples; ++s) {
      const double a = sim[s * sim_stride * n_obs + i];
      const double b = ref[s * ref_stride * n_obs + i];
      num += (a - b) * (a - b);
      den += b * b;
    }
    if (!(den > 0.0)) {
      set_error("observer %d has a zero reference trace", i);
      return FCW_E_ARG;
    }
    sum += std::sqrt(num) / std::sqrt(den);
  }
  *e = sum / n_obs;
  return FCW_OK;
}

fcw_status fcw_query(const fcw_ctx* c, fcw_info* info) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  if (!info) { set_error("null info"); return FCW_E_ARG; }
  std::memset(info, 0, sizeof *info);
  info->ndof = c->ndof;
  info->nnodes = c->nnodes;
  info->ncells = c->ncell_total;
  info->n_cut = c->n_cut;
  info->n_uncut = c->n_uncut;
  info->n_out = c->n_out;
  info->n_loc = c->n_loc;
  info->precision = c->precision;
  info->footprint_bytes = c->footprint;
  info->dt_crit = c->dt_crit;
  info->min_evs_margin = c->min_margin;
  return FCW_OK;
}

fcw_status fcw_export(const fcw_ctx* c, int32_t which, void* dst, int64_t capacity,
                      int64_t* count) {
  g_err.clear();
  fcw_status st = check_ctx(c, 1);
  if (st) return st;
  const void* srcp = nullptr;
  int64_t n = 0;
  size_t es = 8;
  const int64_t ncand = c->n_cut_cand;
  switch (which) {
    case FCW_ARR_CELL_CLASS: srcp = c->d_cls; n = c->ncell_total; es = 1; break;
    case FCW_ARR_CUT_CELLS: srcp = c->d_cut_cells; n = ncand; es = 4; break;
    case FCW_ARR_K_REF: srcp = c->d_kref; n = (int64_t)c->n_loc * c->n_loc; break;
    case FCW_ARR_K_CUT: srcp = c->d_kcut; n = ncand * c->n_loc * c->n_loc; break;
    case FCW_ARR_M_CUT: srcp = c->d_mcut; n = ncand * c->n_s * c->n_s; break;
    case FCW_ARR_LUMPED_CUT: srcp = c->d_lumped; n = ncand * c->n_s; break;
    case FCW_ARR_MASS: srcp = c->d_mass; n = c->state >= 2 ? c->nnodes : 0; break;
    case FCW_ARR_EVS_MARGIN: srcp = c->d_margin; n = ncand; break;
    case FCW_ARR_IMEX_DOFS: srcp = c->d_imex_dofs; n = c->imex_nc > 0 ? c->imex_nc : 0; break;
    default: set_error("unknown array %d", which); return FCW_E_ARG;
  }
  if (count) *count = n;
  if (!dst) return FCW_OK;
  if (capacity < n) {
    set_error("capacity %lld < %lld", (long long)capacity, (long long)n);
    return FCW_E_ARG;
  }
  if (n == 0) return FCW_OK;
  FCW_HIP(hipMemcpyAsync(dst, srcp, (size_t)n * es, hipMemcpyDeviceToHost, c->stream));
  FCW_HIP(hipStreamSynchronize(c->stream));
  return FCW_OK;
}

void fcw_destroy(fcw_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_all(*c);
  delete c;
}

}  // extern "C"
