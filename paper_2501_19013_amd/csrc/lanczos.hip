// Critical time step of the central difference method (paper Sec. 2.3):
//   dt_crit = 2 / sqrt(lambda_max(K, M)),
// with lambda_max the largest eigenvalue of the symmetric operator M^{-1/2} K M^{-1/2}
// on the active DOFs.  FP64 Lanczos iteration on the device (the operator is the tile
// stiffness kernel in FP64, or the B-spline step kernel's stiffness action); the largest eigenvalue theta of the tridiagonal Lanczos
// matrix is found by Sturm-sequence bisection in a one-thread kernel, with the residual
// norm of its Ritz pair.  The iteration stops when that residual is below rtol theta and
// reports theta + residual (Ritz values approach lambda_max from below, so theta alone
// would overestimate dt_crit); it fails with FCW_E_NOCONV when max_iter runs out first.
// Every reduction uses a fixed block count and a fixed tree, so the result is bitwise
// reproducible.
#include <cmath>

#include "common.h"

namespace fcw {

constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

__device__ static double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ static double sum_partials(const double* part, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) v += part[i];
  return block_sum(v, sh);
}

// splitmix64 hash -> uniform in [-1, 1)
__device__ static double hash_unit(uint64_t i) {
  uint64_t z = i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kRedThreads) void start_vector_kernel(double* v, const double* invm,
                                                                    int64_t nnodes, int ncomp,
                                                                    double* part) {
  __shared__ double sh[kRedThreads];
  const int64_t n = nnodes * ncomp;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)kRedBlocks * kRedThreads) {
    const double x = (invm[i % nnodes] > 0.0) ? hash_unit((uint64_t)i) : 0.0;
    v[i] = x;
    s += x * x;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void scale_kernel(double* v, const double* src,
                                                             int64_t n, const double* part,
                                                             double* beta_out) {
  __shared__ double sh[kRedThreads];
  const double nrm = sqrt(sum_partials(part, sh));
  if (blockIdx.x == 0 && threadIdx.x == 0 && beta_out) *beta_out = nrm;
  const double inv = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)kRedBlocks * kRedThreads)
    v[i] = src[i] * inv;
}

__global__ __launch_bounds__(kRedThreads) void dot_kernel(const double* a, const double* b,
                                                           int64_t n, double* part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)kRedBlocks * kRedThreads)
    s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// w <- w - alpha v - beta_prev v_prev, alpha = sum(part); partial sums of |w|^2
__global__ __launch_bounds__(kRedThreads) void axpy_kernel(double* w, const double* v,
                                                            const double* vprev, int64_t n,
                                                            const double* part, double* alpha_out,
                                                            const double* beta_prev,
                                                            double* part2) {
  __shared__ double sh[kRedThreads];
  const double alpha = sum_partials(part, sh);
  const double bp = beta_prev ? *beta_prev : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)kRedBlocks * kRedThreads) {
    double x = w[i] - alpha * v[i];
    if (vprev) x -= bp * vprev[i];
    w[i] = x;
    s += x * x;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

// Largest eigenvalue theta of the symmetric tridiagonal T_k (alpha[0..k), beta[0..k-1)) by
// bisection on the Sturm count, and the last component of its unit eigenvector by inverse
// iteration (Gaussian elimination with partial pivoting on T_k - theta I; work holds 5k
// doubles).  out[0] = theta, out[1] = |s_k|.  With beta_k the next Lanczos coefficient,
// beta_k |s_k| is the residual norm |A y - theta y| of the Ritz pair, so some eigenvalue of
// the operator lies within it of theta.
__host__ __device__ static void tridiag_top(const double* alpha, const double* beta, int k,
                                            double* work, double* out) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    // number of eigenvalues greater than mid
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
      const double b2 = (i > 0) ? beta[i - 1] * beta[i - 1] : 0.0;
      q = alpha[i] - mid - ((i > 0) ? b2 / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q > 0.0) ++cnt;
    }
    if (cnt >= 1) lo = mid; else hi = mid;
  }
  const double theta = lo;
  out[0] = theta;
  // inverse iteration: (T - theta I) x_{n+1} = x_n, by Gaussian elimination with row
  // interchanges; the rows of U hold u0 (diagonal), u1, u2 (first and second
  // super-diagonals), ml the multipliers, sw whether rows i, i+1 were interchanged
  double* u0 = work;
  double* u1 = work + k;
  double* u2 = work + 2 * k;
  double* ml = work + 3 * k;
  double* sw = work + 4 * k;
  double* x = work + 5 * k;
  double scale = 0.0;
  for (int i = 0; i < k; ++i)
    scale = fmax(scale, fabs(alpha[i] - theta) + (i < k - 1 ? fabs(beta[i]) : 0.0));
  const double tiny = (scale > 0.0 ? scale : 1.0) * 1e-290;
  // the current row holds d at column i and e at column i + 1
  double d = alpha[0] - theta, e = (k > 1) ? beta[0] : 0.0;
  for (int i = 0; i < k - 1; ++i) {
    const double b = beta[i];                // row i+1 at column i
    const double dn = alpha[i + 1] - theta;  // row i+1 at column i+1
    const double en = (i + 1 < k - 1) ? beta[i + 1] : 0.0;  // row i+1 at column i+2
    if (fabs(d) >= fabs(b)) {
      const double dd = (d != 0.0) ? d : tiny;
      const double m = b / dd;
      u0[i] = dd; u1[i] = e; u2[i] = 0.0; ml[i] = m; sw[i] = 0.0;
      d = dn - m * e;
      e = en;
    } else {
      const double m = d / b;
      u0[i] = b; u1[i] = dn; u2[i] = en; ml[i] = m; sw[i] = 1.0;
      d = e - m * dn;
      e = -m * en;
    }
  }
  u0[k - 1] = (d != 0.0) ? d : tiny;
  u1[k - 1] = 0.0;
  u2[k - 1] = 0.0;
  for (int i = 0; i < k; ++i) x[i] = 1.0;
  for (int rep = 0; rep < 3; ++rep) {
    for (int i = 0; i < k - 1; ++i) {
      if (sw[i] != 0.0) {
        const double t = x[i];
        x[i] = x[i + 1];
        x[i + 1] = t - ml[i] * x[i];
      } else {
        x[i + 1] -= ml[i] * x[i];
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double v = x[i];
      if (i + 1 < k) v -= u1[i] * x[i + 1];
      if (i + 2 < k) v -= u2[i] * x[i + 2];
      x[i] = v / u0[i];
    }
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm = fmax(nrm, fabs(x[i]));
    if (!(nrm > 0.0) || !(nrm < INFINITY)) break;
    for (int i = 0; i < k; ++i) x[i] /= nrm;
  }
  double n2 = 0.0;
  for (int i = 0; i < k; ++i) n2 += x[i] * x[i];
  out[1] = (n2 > 0.0 && n2 < INFINITY) ? fabs(x[k - 1]) / sqrt(n2) : 1.0;
}

__global__ void tridiag_max_kernel(const double* alpha, const double* beta, int k, double* work,
                                   double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tridiag_top(alpha, beta, k, work, out);
}

fcw_status lanczos_run(const LanczosOp& op, int max_iter, double rtol, double* lmax) {
  const int64_t n = op.n;
  const hipStream_t stream = op.stream;
  double *v0 = nullptr, *v1 = nullptr, *w = nullptr, *ab = nullptr, *part = nullptr;
  const size_t vb = (size_t)n * sizeof(double);
  FCW_HIP(hipMallocAsync((void**)&v0, vb, stream));
  FCW_HIP(hipMallocAsync((void**)&v1, vb, stream));
  FCW_HIP(hipMallocAsync((void**)&w, vb, stream));
  // alpha, beta, two result words, the tridiagonal solver's work (6 max_iter)
  FCW_HIP(hipMallocAsync((void**)&ab, (8 * (size_t)max_iter + 2) * sizeof(double), stream));
  FCW_HIP(hipMallocAsync((void**)&part, 2 * kRedBlocks * sizeof(double), stream));
  double* alpha = ab;
  double* beta = ab + max_iter;
  double* res = ab + 2 * max_iter;
  double* twork = ab + 2 * max_iter + 2;
  double* part2 = part + kRedBlocks;

  start_vector_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(w, op.mask, op.nmask, op.ncomp,
                                                                  part);
  scale_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(v1, w, n, part, nullptr);
  FCW_HIP(hipGetLastError());
  double* vcur = v1;
  double* vprev = v0;
  double theta = 0.0, resid = INFINITY;
  bool converged = false;
  const int check = 20;
  fcw_status st = FCW_OK;
  for (int j = 0; j < max_iter; ++j) {
    st = op.apply(op.arg, vcur, w);
    if (st != FCW_OK) break;
    dot_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(w, vcur, n, part);
    axpy_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(
        w, vcur, j > 0 ? vprev : nullptr, n, part, alpha + j, j > 0 ? beta + j - 1 : nullptr,
        part2);
    scale_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(vprev, w, n, part2, beta + j);
    FCW_HIP(hipGetLastError());
    double* t = vprev;
    vprev = vcur;
    vcur = t;
    const int k = j + 1;
    if (k % check == 0 || k == max_iter) {
      tridiag_max_kernel<<<1, 64, 0, stream>>>(alpha, beta, k, twork, res);
      double hb[3];
      FCW_HIP(hipMemcpyAsync(&hb[0], res, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
      FCW_HIP(hipMemcpyAsync(&hb[2], beta + j, sizeof(double), hipMemcpyDeviceToHost, stream));
      FCW_HIP(hipStreamSynchronize(stream));
      theta = hb[0];
      // residual norm of the Ritz pair: beta_k |s_k|
      resid = fabs(hb[2]) * hb[1];
      if (theta > 0.0 && resid <= rtol * theta) {
        converged = true;
        break;
      }
      if (!(hb[2] > 1e-300 * fabs(theta))) {  // invariant subspace: theta is exact
        resid = 0.0;
        converged = true;
        break;
      }
    }
  }
  FCW_HIP(hipFreeAsync(v0, stream));
  FCW_HIP(hipFreeAsync(v1, stream));
  FCW_HIP(hipFreeAsync(w, stream));
  FCW_HIP(hipFreeAsync(ab, stream));
  FCW_HIP(hipFreeAsync(part, stream));
  FCW_HIP(hipStreamSynchronize(stream));
  if (st != FCW_OK) return st;
  if (!(theta > 0.0) || !std::isfinite(theta)) {
    set_error("Lanczos iteration gave no positive eigenvalue (%g)", theta);
    return FCW_E_NOCONV;
  }
  if (!converged) {
    set_error("Lanczos: residual %.3e of the largest Ritz value %.10e above rtol after %d "
              "iterations", resid / theta, theta, max_iter);
    return FCW_E_NOCONV;
  }
  // theta rises toward lambda_max from below; theta + residual bounds from above the
  // eigenvalue it approximates, so the step derived from it errs on the safe side
  *lmax = theta + resid;
  return FCW_OK;
}

static fcw_status apply_scaled_ctx(void* arg, const double* v, double* w) {
  return launch_apply_scaled64(*(Ctx*)arg, v, w);
}

fcw_status lanczos_lambda_max(Ctx& c, int max_iter, double rtol, double* lmax) {
  LanczosOp op{c.stream, c.ndof, c.d_invm64, c.nnodes, c.ncomp, apply_scaled_ctx, &c};
  return lanczos_run(op, max_iter, rtol, lmax);
}

}  // namespace fcw
