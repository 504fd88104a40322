// Observation of a run (fcw_run): receiver traces after every step, growth checks of the
// increments and the discrete energy of the central difference scheme.
//
//  * Trace of receiver r (Sec. 3.2, observer traces): u_h(x_r) = sum_a N_a(x_r) u_a over
//    the nodes a of the cell holding x_r, per component, summed in FP64 by one wave in a
//    fixed butterfly order (bitwise reproducible).  One small launch per step samples the
//    state the step just wrote, for every problem, right-hand side and receiver.
//  * Sums over the DOFs per right-hand side with a fixed block count and a fixed tree:
//    sum d_i^2 for the growth checks; sum m_i d_i^2, u.Ku and d.Ku for the discrete energy
//    E_{k+1/2} = 1/2 v^T M v + 1/2 u_{k+1}^T K u_k with v = d_{k+1} / dt and
//    u_k = u_{k+1} - d_{k+1}, i.e. E = 1/2 (d^T M d / dt^2 + u^T K u - d^T K u) (K symmetric).
#include <algorithm>
#include <cstring>

#include "step_common.h"

namespace fcw {

namespace {

constexpr int kSumBlocks = 256;
constexpr int kSumThreads = 256;
constexpr int kMaxTargets = 16;  // trace targets per launch (passed by value)

struct TraceArg {
  const void* ua;
  const void* ub;
  const RecDev* rec;
  double* traces;
  int64_t tlen, k0, nnodes;
  int nrhs, nsteps, nrec, ncomp, p, dim;
  int np[3];
};

struct TraceLaunch {
  TraceArg t[kMaxTargets];
  int n;
};

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// grid (nrec_max, nrhs_max, targets); j < 0: sample the state of the call's start
template <typename T>
__global__ __launch_bounds__(64) void trace_kernel(TraceLaunch L, int j) {
  const int ti = blockIdx.z;
  if (ti >= L.n) return;
  const TraceArg& a = L.t[ti];
  const int r = blockIdx.x, rhs = blockIdx.y;
  if (r >= a.nrec || rhs >= a.nrhs) return;
  if (j >= a.nsteps) return;  // this problem has finished its steps
  // the state after step j of a call of nsteps steps sits in u when nsteps - 1 - j is even
  const T* base = (const T*)((j < 0 || ((a.nsteps - 1 - j) & 1) == 0) ? a.ua : a.ub);
  const T* u = base + (int64_t)rhs * a.ncomp * a.nnodes;
  const RecDev& rd = a.rec[r];
  const int np1 = a.p + 1;
  const int ns = (a.dim == 3) ? np1 * np1 * np1 : np1 * np1;
  const int lane = threadIdx.x;
  const int64_t row = a.k0 + j + 1;
  double* out = a.traces + (((int64_t)rhs * a.tlen + row) * a.nrec + r) * a.ncomp;
  for (int comp = 0; comp < a.ncomp; ++comp) {
    double s = 0.0;
    for (int loc = lane; loc < ns; loc += 64) {
      const int ix = loc % np1, iy = (loc / np1) % np1, iz = loc / (np1 * np1);
      const int64_t gx = (int64_t)rd.cell[0] * a.p + ix;
      const int64_t gy = (int64_t)rd.cell[1] * a.p + iy;
      const int64_t gz = (a.dim == 3) ? (int64_t)rd.cell[2] * a.p + iz : 0;
      const int64_t node = gx + (int64_t)a.np[0] * (gy + (int64_t)a.np[1] * gz);
      s += rd.w[loc] * (double)u[comp * a.nnodes + node];
    }
    s = wave_sum(s);
    if (lane == 0) out[comp] = s;
  }
}

// Partial sums over the DOFs of right-hand side blockIdx.y (see the file comment).
template <typename T, bool ENERGY>
__global__ __launch_bounds__(kSumThreads) void sums_kernel(const T* u, const T* d, const T* r,
                                                           const double* invm64, int64_t nnodes,
                                                           int64_t ndof, double* part) {
  __shared__ double sh[3][kSumThreads];
  const int rhs = blockIdx.y;
  const int64_t off = (int64_t)rhs * ndof;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kSumThreads + threadIdx.x; i < ndof;
       i += (int64_t)kSumBlocks * kSumThreads) {
    const double dv = (double)d[off + i];
    if (ENERGY) {
      const double im = invm64[i % nnodes];
      const double m = (im > 0.0) ? 1.0 / im : 0.0;
      const double kv = (double)r[off + i];
      s0 += m * dv * dv;
      s1 += (double)u[off + i] * kv;
      s2 += dv * kv;
    } else {
      s0 += dv * dv;
    }
  }
  const int t = threadIdx.x;
  sh[0][t] = s0;
  sh[1][t] = s1;
  sh[2][t] = s2;
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + w];
    __syncthreads();
  }
  if (t < 3) part[((int64_t)rhs * 3 + t) * kSumBlocks + blockIdx.x] = sh[t][0];
}

// totals[rhs * 3 + q] = sum over the blocks' partial sums, fixed order
__global__ __launch_bounds__(kSumThreads) void sums_final_kernel(const double* part,
                                                                 double* totals) {
  __shared__ double sh[kSumThreads];
  const int k = blockIdx.x;  // rhs * 3 + q
  const int t = threadIdx.x;
  double v = 0.0;
  for (int i = t; i < kSumBlocks; i += kSumThreads) v += part[(int64_t)k * kSumBlocks + i];
  sh[t] = v;
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) totals[k] = sh[0];
}

// d[rhs][dof] += coef * M^{-1} f_t(t) b for the volumetric load entries of each
// right-hand side (grid: entries x right-hand sides)
template <typename T>
__global__ void gauss_apply_kernel(const int64_t* dof, const double* val, const int32_t* off,
                                   const SourceDev* src, const double* invm64, int64_t nnodes,
                                   int64_t ndof, double t, double coef, T* d) {
  const int rhs = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = off[rhs + 1] - off[rhs];
  if (i >= n) return;
  const int64_t e = off[rhs] + i;
  const int64_t g = dof[e];
  const double f = coef * invm64[g % nnodes] * ricker(t, src[rhs].f0) * val[e];
  T* dp = d + (int64_t)rhs * ndof + g;
  *dp = (T)((double)*dp + f);
}

}  // namespace

fcw_status launch_gauss_loads(hipStream_t s, const LoadTarget* t, int n, int j) {
  for (int i = 0; i < n; ++i) {
    const LoadTarget& x = t[i];
    const Ctx& c = *x.ctx;
    // the load of step j + 1 enters the increment after step j; none after the last step
    const int k = j + 1;
    if (k >= x.nsteps || !c.g_active) continue;
    int64_t nmax = 0;
    for (int r = 0; r < x.nrhs; ++r) nmax = std::max<int64_t>(nmax, c.g_off[r + 1] - c.g_off[r]);
    if (nmax == 0) continue;
    const double coef = (x.start && k == 0) ? 0.5 * x.dt * x.dt : x.dt * x.dt;
    const dim3 grid((unsigned)((nmax + 255) / 256), x.nrhs);
    const double tk = x.t0 + k * x.dt;
    if (c.precision == FCW_FP64)
      gauss_apply_kernel<double><<<grid, 256, 0, s>>>(c.d_gdof, c.d_gval, c.d_goff, c.d_src,
                                                      c.d_invm64, c.nnodes, c.ndof, tk, coef,
                                                      (double*)x.d);
    else
      gauss_apply_kernel<float><<<grid, 256, 0, s>>>(c.d_gdof, c.d_gval, c.d_goff, c.d_src,
                                                     c.d_invm64, c.nnodes, c.ndof, tk, coef,
                                                     (float*)x.d);
    FCW_HIP(hipGetLastError());
  }
  return FCW_OK;
}

fcw_status launch_traces(hipStream_t s, const TraceTarget* t, int n, int j) {
  for (int base = 0; base < n; base += kMaxTargets) {
    TraceLaunch L;
    std::memset(&L, 0, sizeof L);
    L.n = std::min(kMaxTargets, n - base);
    int maxrec = 1, maxrhs = 1;
    bool fp64 = true;
    for (int i = 0; i < L.n; ++i) {
      const TraceTarget& x = t[base + i];
      const Ctx& c = *x.ctx;
      TraceArg& a = L.t[i];
      a.ua = x.u;
      a.ub = x.ub;
      a.rec = c.d_rec;
      a.traces = x.traces;
      a.tlen = x.tlen;
      a.k0 = x.k0;
      a.nnodes = c.nnodes;
      a.nrhs = x.nrhs;
      a.nsteps = x.nsteps;
      a.nrec = x.nrec;
      a.ncomp = c.ncomp;
      a.p = c.p;
      a.dim = c.dim;
      for (int k = 0; k < 3; ++k) a.np[k] = c.npts[k];
      maxrec = std::max(maxrec, x.nrec);
      maxrhs = std::max(maxrhs, x.nrhs);
      fp64 = c.precision == FCW_FP64;  // every target of one launch shares the precision
    }
    const dim3 grid(maxrec, maxrhs, L.n);
    if (fp64) trace_kernel<double><<<grid, 64, 0, s>>>(L, j);
    else trace_kernel<float><<<grid, 64, 0, s>>>(L, j);
    FCW_HIP(hipGetLastError());
  }
  return FCW_OK;
}

fcw_status state_sums(Ctx& c, hipStream_t s, int nrhs, const void* u, const void* d,
                      const void* r, bool energy) {
  if (nrhs < 1 || nrhs > 64) {
    set_error("state sums need 1 <= nrhs <= 64");
    return FCW_E_ARG;
  }
  if (!c.d_red) {
    const size_t bytes = (size_t)64 * 3 * (kSumBlocks + 1) * sizeof(double);
    FCW_HIP(hipMalloc((void**)&c.d_red, bytes));
    c.footprint += (int64_t)bytes;
    FCW_HIP(hipHostMalloc((void**)&c.h_red, 64 * 3 * sizeof(double), hipHostMallocDefault));
  }
  double* part = c.d_red;
  double* totals = c.d_red + (size_t)64 * 3 * kSumBlocks;
  const dim3 grid(kSumBlocks, nrhs);
  if (c.precision == FCW_FP64) {
    if (energy)
      sums_kernel<double, true><<<grid, kSumThreads, 0, s>>>(
          (const double*)u, (const double*)d, (const double*)r, c.d_invm64, c.nnodes, c.ndof,
          part);
    else
      sums_kernel<double, false><<<grid, kSumThreads, 0, s>>>(
          nullptr, (const double*)d, nullptr, c.d_invm64, c.nnodes, c.ndof, part);
  } else {
    if (energy)
      sums_kernel<float, true><<<grid, kSumThreads, 0, s>>>(
          (const float*)u, (const float*)d, (const float*)r, c.d_invm64, c.nnodes, c.ndof,
          part);
    else
      sums_kernel<float, false><<<grid, kSumThreads, 0, s>>>(
          nullptr, (const float*)d, nullptr, c.d_invm64, c.nnodes, c.ndof, part);
  }
  FCW_HIP(hipGetLastError());
  sums_final_kernel<<<nrhs * 3, kSumThreads, 0, s>>>(part, totals);
  FCW_HIP(hipGetLastError());
  FCW_HIP(hipMemcpyAsync(c.h_red, totals, (size_t)nrhs * 3 * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  FCW_HIP(hipStreamSynchronize(s));
  return FCW_OK;
}

}  // namespace fcw
