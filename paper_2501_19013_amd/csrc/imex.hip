// Newmark IMEX (paper Sec. 2.5, Alg. imex) on the device, FP64.
//
// The DOFs split by the support of their basis functions: a node of at least one cut
// cell is implicit ("c"), every other active node explicit ("d").  Uncut cells have a
// diagonal (GLL) mass, so M = diag(M^dd, M^cc), M^cc the consistent mass of the cut DOFs
// (original tree-integrated cut-cell masses M^o_e, no stabilisation, plus the uncut
// cells' GLL diagonals).  One step:
//
//   1. explicit DOFs: the central-difference step of the explicit solver (its tile and
//      cut-cell kernels; the values it leaves on implicit DOFs are replaced below);
//   2. implicit predictors u_p = u_k + dt v_k + (1/2 - beta) dt^2 a_k on the implicit
//      DOFs, the explicit DOFs' new values serving as theirs;
//   3. r = K u_p (the explicit solver's stiffness action);
//   4. S a_{k+1} = F_{k+1} - r on the implicit DOFs, S = M^cc + beta dt^2 K^cc: a dense
//      product with S^{-1}, formed once from the Cholesky factor of S (forward and
//      backward sweeps against the unit vectors, one workgroup per column);
//   5. v_{k+1} = v_k + dt ((1 - gamma) a_k + gamma a_{k+1}),
//      u_{k+1} = u_p + beta dt^2 a_{k+1}.
//
// The same set-up serves central differences with the consistent cut-DOF mass (the
// consistent-mass spectral cell method, eq. cdm with M = diag(M^dd, M^cc)): per step
// a = (M^cc)^{-1} (F_k - K u_k) on the implicit DOFs, the lumped step elsewhere.
//
// S and M^cc are assembled dense (entry by entry from the cells around the two nodes,
// in a fixed order) and factored on the device by a blocked right-looking Cholesky.
// The dense form bounds the implicit set (FCW_IMEX_MAX_NC); a sparse factorisation is
// what large cut fractions would need.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "step_common.h"

namespace fcw {

constexpr double kBeta = 0.25, kGamma = 0.5;
constexpr int kCholNb = 32;

// ---- implicit set ----

// mark[node] = 1 for the nodes of every kept cut cell
__global__ void imex_mark_kernel(const int32_t* info, const int32_t* cut_cells, int64_t ncand,
                                 int dim, int p, int n0, int n1, int np0, int np1,
                                 int32_t* mark) {
  const int np1p = p + 1;
  const int ns = (dim == 3) ? np1p * np1p * np1p : np1p * np1p;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncand * ns) return;
  const int64_t q = t / ns;
  const int loc = (int)(t % ns);
  const int cell = cut_cells[q];
  if (info[cell] != (int32_t)q) return;  // reclassified OUT
  const int cx = cell % n0, cy = (cell / n0) % n1, cz = cell / (n0 * n1);
  const int i0 = loc % np1p, i1 = (loc / np1p) % np1p, i2 = loc / (np1p * np1p);
  const int64_t node = (int64_t)(cx * p + i0) +
                       (int64_t)np0 * ((cy * p + i1) + (int64_t)np1 * (dim == 3 ? cz * p + i2 : 0));
  mark[node] = 1;
}

__global__ void imex_dofs_kernel(const int32_t* mark, const int32_t* pos, int64_t nnodes,
                                 int64_t ncn, int ncomp, int64_t* dofs) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nnodes || !mark[node]) return;
  for (int k = 0; k < ncomp; ++k) dofs[k * ncn + pos[node]] = k * nnodes + node;
}

// ---- dense S and M^cc, entry by entry ----

struct ImexAsm {
  const int64_t* dofs;
  const int32_t* info;
  const double* kref;   // [nl][nl]
  const double* lref;   // [ns]
  const double* kcut;   // [ncand][nl][nl]
  const double* mcut;   // [ncand][ns][ns]
  double* S;            // [nc][nc]
  double* M;            // [nc][nc]
  int64_t nc, nnodes;
  int dim, p, ns, nl;
  int n[3], np[3];
  double bdt2;          // beta dt^2
};

__global__ void imex_assemble_kernel(ImexAsm a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
  if (i >= a.nc || j >= a.nc) return;
  const int64_t gi = a.dofs[i], gj = a.dofs[j];
  const int ci = (int)(gi / a.nnodes), cj = (int)(gj / a.nnodes);
  const int64_t ni = gi % a.nnodes, nj = gj % a.nnodes;
  int xi[3], xj[3];
  xi[0] = (int)(ni % a.np[0]); xi[1] = (int)((ni / a.np[0]) % a.np[1]);
  xi[2] = (int)(ni / ((int64_t)a.np[0] * a.np[1]));
  xj[0] = (int)(nj % a.np[0]); xj[1] = (int)((nj / a.np[0]) % a.np[1]);
  xj[2] = (int)(nj / ((int64_t)a.np[0] * a.np[1]));
  double ks = 0.0, ms = 0.0;
  bool near = true;
  for (int k = 0; k < a.dim; ++k)
    if (abs(xi[k] - xj[k]) > a.p) near = false;
  if (near) {
    // the cells around node i, in a fixed order; those that also hold node j contribute
    const int nz = (a.dim == 3) ? 2 : 1;
    for (int sz = 0; sz < nz; ++sz)
      for (int sy = 0; sy < 2; ++sy)
        for (int sx = 0; sx < 2; ++sx) {
          const int sel[3] = {sx, sy, sz};
          int cc[3] = {0, 0, 0};
          bool ok = true;
          for (int k = 0; k < a.dim; ++k) {
            // candidate cells along axis k: floor(x/p) and, on a cell boundary, floor(x/p)-1
            const int cand = (sel[k] == 0) ? xi[k] / a.p : xi[k] / a.p - 1;
            if (sel[k] == 1 && xi[k] % a.p != 0) ok = false;
            if (cand < 0 || cand >= a.n[k]) ok = false;
            if (xj[k] < cand * a.p || xj[k] > cand * a.p + a.p) ok = false;
            cc[k] = cand;
          }
          if (!ok) continue;
          const int64_t cell = cc[0] + (int64_t)a.n[0] * (cc[1] + (int64_t)a.n[1] * cc[2]);
          const int inf = a.info[cell];
          if (inf == kInfoOut) continue;
          const int np1 = a.p + 1;
          const int li = (xi[0] - cc[0] * a.p) + np1 * ((xi[1] - cc[1] * a.p) +
                                                         np1 * (a.dim == 3 ? xi[2] - cc[2] * a.p : 0));
          const int lj = (xj[0] - cc[0] * a.p) + np1 * ((xj[1] - cc[1] * a.p) +
                                                         np1 * (a.dim == 3 ? xj[2] - cc[2] * a.p : 0));
          const int ri = ci * a.ns + li, rj = cj * a.ns + lj;
          if (inf >= 0) {
            ks += a.kcut[((int64_t)inf * a.nl + ri) * a.nl + rj];
            if (ci == cj) ms += a.mcut[((int64_t)inf * a.ns + li) * a.ns + lj];
          } else {
            ks += a.kref[(int64_t)ri * a.nl + rj];
            if (ci == cj && li == lj) ms += a.lref[li];
          }
        }
  }
  a.M[i * a.nc + j] = ms;
  a.S[i * a.nc + j] = ms + a.bdt2 * ks;
}

// ---- blocked right-looking Cholesky, lower, row-major, in place ----

// factor the nb x nb diagonal block at k0 (one workgroup)
__global__ __launch_bounds__(256) void chol_diag_kernel(double* A, int64_t n, int64_t k0, int nb,
                                                        int32_t* flag) {
  __shared__ double L[kCholNb][kCholNb + 1];
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += 256) L[e / nb][e % nb] = A[(k0 + e / nb) * n + k0 + e % nb];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t == 0) {
      const double d = L[j][j];
      if (!(d > 0.0)) flag[0] = 1;
      L[j][j] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    for (int i = j + 1 + t; i < nb; i += 256) L[i][j] /= L[j][j];
    __syncthreads();
    for (int e = t; e < nb * nb; e += 256) {
      const int i = e / nb, k = e % nb;
      if (i > j && k > j && k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    A[(k0 + i) * n + k0 + k] = (k <= i) ? L[i][k] : 0.0;
  }
}

// rows below the diagonal block: L21 = A21 L11^{-T} (one thread per row)
__global__ __launch_bounds__(256) void chol_panel_kernel(double* A, int64_t n, int64_t k0, int nb) {
  __shared__ double L[kCholNb][kCholNb + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256)
    L[e / nb][e % nb] = A[(k0 + e / nb) * n + k0 + e % nb];
  __syncthreads();
  const int64_t i = k0 + nb + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x[kCholNb];
  for (int j = 0; j < nb; ++j) {
    double s = A[i * n + k0 + j];
    for (int m = 0; m < j; ++m) s -= x[m] * L[j][m];
    x[j] = s / L[j][j];
  }
  for (int j = 0; j < nb; ++j) A[i * n + k0 + j] = x[j];
}

// trailing update A22 -= L21 L21^T on the lower triangle, 32 x 32 tiles
__global__ __launch_bounds__(256) void chol_update_kernel(double* A, int64_t n, int64_t k0, int nb) {
  const int64_t r0 = k0 + nb;
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double Pi[kCholNb][kCholNb + 1], Pj[kCholNb][kCholNb + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kCholNb * nb; e += 256) {
    const int r = e / nb, m = e % nb;
    const int64_t gi = r0 + ti * kCholNb + r, gj = r0 + tj * kCholNb + r;
    Pi[r][m] = gi < n ? A[gi * n + k0 + m] : 0.0;
    Pj[r][m] = gj < n ? A[gj * n + k0 + m] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < kCholNb * kCholNb; e += 256) {
    const int r = e / kCholNb, q = e % kCholNb;
    const int64_t gi = r0 + ti * kCholNb + r, gj = r0 + tj * kCholNb + q;
    if (gi >= n || gj >= n || gj > gi) continue;
    double s = 0.0;
    for (int m = 0; m < nb; ++m) s += Pi[r][m] * Pj[q][m];
    A[gi * n + gj] -= s;
  }
}

__global__ void transpose_kernel(const double* A, double* B, int64_t n) {
  __shared__ double tile[32][33];
  const int64_t x0 = (int64_t)blockIdx.x * 32, y0 = (int64_t)blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int64_t y = y0 + r, x = x0 + threadIdx.x;
    tile[r][threadIdx.x] = (y < n && x < n) ? A[y * n + x] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int64_t y = x0 + r, x = y0 + threadIdx.x;
    if (y < n && x < n) B[y * n + x] = tile[threadIdx.x][r];
  }
}

static fcw_status cholesky(Ctx& c, double* A, double* At, int64_t n) {
  FCW_HIP(hipMemsetAsync(c.d_imex_flag, 0, sizeof(int32_t), c.stream));
  for (int64_t k0 = 0; k0 < n; k0 += kCholNb) {
    const int nb = (int)std::min<int64_t>(kCholNb, n - k0);
    chol_diag_kernel<<<1, 256, 0, c.stream>>>(A, n, k0, nb, c.d_imex_flag);
    const int64_t rest = n - k0 - nb;
    if (rest > 0) {
      chol_panel_kernel<<<(unsigned)((rest + 255) / 256), 256, 0, c.stream>>>(A, n, k0, nb);
      const unsigned nt = (unsigned)((rest + kCholNb - 1) / kCholNb);
      chol_update_kernel<<<dim3(nt, nt), 256, 0, c.stream>>>(A, n, k0, nb);
    }
  }
  FCW_HIP(hipGetLastError());
  const unsigned nt = (unsigned)((n + 31) / 32);
  transpose_kernel<<<dim3(nt, nt), dim3(32, 8), 0, c.stream>>>(A, At, n);
  FCW_HIP(hipGetLastError());
  int32_t bad = 0;
  FCW_HIP(hipMemcpyAsync(&bad, c.d_imex_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  if (bad) {
    set_error("IMEX: the implicit-DOF matrix is not positive definite");
    return FCW_E_NOCONV;
  }
  return FCW_OK;
}

// ---- x = A^{-1} b with A = L L^T: one workgroup per right-hand side, x in LDS ----
// L row-major lower (rows contiguous), Lt = L^T row-major (rows of L^T contiguous).
__global__ __launch_bounds__(256) void chol_solve_kernel(const double* L, const double* Lt,
                                                         int64_t n, const double* b, double* x) {
  extern __shared__ double xs[];
  const int r = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double* br = b + (int64_t)r * n;
  for (int64_t i = t; i < n; i += 256) xs[i] = br[i];
  __syncthreads();
  // forward: L y = b, 32 rows at a time; each wave reduces rows against the solved part
  for (int64_t r0 = 0; r0 < n; r0 += 32) {
    const int nb = (int)min((int64_t)32, n - r0);
    for (int q = wave; q < nb; q += 4) {
      const int64_t i = r0 + q;
      double s = 0.0;
      for (int64_t j = lane; j < r0; j += 64) s += L[i * n + j] * xs[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) xs[i] -= s;
    }
    __syncthreads();
    if (wave == 0) {
      for (int m = 0; m < nb; ++m) {
        if (lane == 0) xs[r0 + m] /= L[(r0 + m) * n + r0 + m];
        __builtin_amdgcn_wave_barrier();
        const double ym = xs[r0 + m];
        if (lane > m && lane < nb) xs[r0 + lane] -= L[(r0 + lane) * n + r0 + m] * ym;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  // backward: L^T x = y, 32 rows at a time from the bottom
  for (int64_t r1 = n; r1 > 0; r1 -= 32) {
    const int64_t r0 = max((int64_t)0, r1 - 32);
    const int nb = (int)(r1 - r0);
    for (int q = wave; q < nb; q += 4) {
      const int64_t i = r0 + q;
      double s = 0.0;
      for (int64_t j = r1 + lane; j < n; j += 64) s += Lt[i * n + j] * xs[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) xs[i] -= s;
    }
    __syncthreads();
    if (wave == 0) {
      for (int m = nb - 1; m >= 0; --m) {
        if (lane == 0) xs[r0 + m] /= Lt[(r0 + m) * n + r0 + m];
        __builtin_amdgcn_wave_barrier();
        const double xm = xs[r0 + m];
        if (lane < m) xs[r0 + lane] -= Lt[(r0 + lane) * n + r0 + m] * xm;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  double* xr = x + (int64_t)r * n;
  for (int64_t i = t; i < n; i += 256) xr[i] = xs[i];
}

// x_r = A b_r for every right-hand side r, A dense symmetric n x n (row-major): one wave
// per row, each row read once for up to 8 right-hand sides
__global__ __launch_bounds__(256) void sym_gemv_kernel(const double* A, int64_t n, const double* b,
                                                       double* x, int nrhs) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* row = A + i * n;
  for (int r0 = 0; r0 < nrhs; r0 += 8) {
    const int nr = min(8, nrhs - r0);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t j = lane; j < n; j += 64) {
      const double aij = row[j];
  #pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nr) acc[q] += aij * b[(int64_t)(r0 + q) * n + j];
    }
  #pragma unroll
    for (int q = 0; q < 8; ++q) {
      double v = acc[q];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (q < nr && lane == 0) x[(int64_t)(r0 + q) * n + i] = v;
    }
  }
}

// the same for one right-hand side: 16-byte loads of the row and of b, two rows per wave
// pass in flight (n even: rows start 16-byte aligned)
__global__ __launch_bounds__(256) void sym_gemv1_kernel(const double* A, int64_t n,
                                                        const double* b, double* x) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double2* row = (const double2*)(A + i * n);
  const double2* bv = (const double2*)b;
  const int64_t n2 = n / 2;
  double acc0 = 0.0, acc1 = 0.0;
  int64_t j = lane;
  for (; j + 64 < n2; j += 128) {
    const double2 a0 = row[j], a1 = row[j + 64];
    const double2 b0 = bv[j], b1 = bv[j + 64];
    acc0 += a0.x * b0.x + a0.y * b0.y;
    acc1 += a1.x * b1.x + a1.y * b1.y;
  }
  if (j < n2) {
    const double2 a0 = row[j], b0 = bv[j];
    acc0 += a0.x * b0.x + a0.y * b0.y;
  }
  double v = acc0 + acc1;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) x[i] = v;
}

__global__ void identity_kernel(double* A, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * n) A[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// ---- per-step vector kernels over [nrhs][nc] ----

__global__ void imex_gather_kernel(const double* u, const int64_t* dofs, int64_t nc, int64_t ndof,
                                   int nrhs, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nrhs) return;
  const int64_t r = t / nc, i = t % nc;
  out[t] = u[r * ndof + dofs[i]];
}

// u[c] = u_k + dt v + (1/2 - beta) dt^2 a
__global__ void imex_predict_kernel(double* u, const int64_t* dofs, const double* uold,
                                    const double* v, const double* a, int64_t nc, int64_t ndof,
                                    int nrhs, double dt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nrhs) return;
  const int64_t r = t / nc, i = t % nc;
  u[r * ndof + dofs[i]] = uold[t] + dt * v[t] + (0.5 - kBeta) * dt * dt * a[t];
}

// b = F(t) - r on the implicit DOFs (F from the point sources of the call)
__global__ void imex_rhs_kernel(const double* rk, const int64_t* dofs, const SourceDev* src,
                                int64_t nc, int64_t ndof, int64_t nnodes, int nrhs, int dim, int p,
                                int np0, int np1, double t, double* b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * nrhs) return;
  const int64_t r = e / nc, i = e % nc;
  const int64_t g = dofs[i];
  double f = 0.0;
  if (src) {
    const SourceDev& s = src[r];
    const int comp = (int)(g / nnodes);
    const int64_t node = g % nnodes;
    const int x = (int)(node % np0), y = (int)((node / np0) % np1), z = (int)(node / ((int64_t)np0 * np1));
    const int sx = x - s.cell[0] * p, sy = y - s.cell[1] * p, sz = (dim == 3) ? z - s.cell[2] * p : 0;
    const int np1p = p + 1;
    const int ns = (dim == 3) ? np1p * np1p * np1p : np1p * np1p;
    if (sx >= 0 && sx <= p && sy >= 0 && sy <= p && sz >= 0 && sz <= p)
      f = ricker(t, s.f0) * s.b[comp * ns + sx + np1p * (sy + np1p * sz)];
  }
  b[e] = f - rk[r * ndof + g];
}

// v += dt ((1 - gamma) a_k + gamma a_{k+1}); u[c] += beta dt^2 a_{k+1}; d[c] = u[c] - u_k;
// a = a_{k+1}
__global__ void imex_correct_kernel(double* u, double* d, const int64_t* dofs, const double* uold,
                                    double* v, double* a, const double* anew, int64_t nc,
                                    int64_t ndof, int nrhs, double dt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nrhs) return;
  const int64_t r = t / nc, i = t % nc;
  const int64_t g = r * ndof + dofs[i];
  const double an = anew[t];
  v[t] = v[t] + dt * ((1.0 - kGamma) * a[t] + kGamma * an);
  const double un = u[g] + kBeta * dt * dt * an;
  u[g] = un;
  d[g] = un - uold[t];
  a[t] = an;
}

// consistent-mass central differences on the implicit DOFs: d = d_k + w a, u = u_k + d
__global__ void cons_fix_kernel(double* u, double* d, const int64_t* dofs, const double* uold,
                                const double* dold, const double* a, int64_t nc, int64_t ndof,
                                int nrhs, double w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nrhs) return;
  const int64_t r = t / nc, i = t % nc;
  const int64_t g = r * ndof + dofs[i];
  const double dn = dold[t] + w * a[t];
  d[g] = dn;
  u[g] = uold[t] + dn;
}

// x = A b for nrhs right-hand sides (A the dense inverse of S or M^cc)
static void solve_product(Ctx& c, const double* A, int64_t n, const double* b, double* x,
                          int nrhs) {
  if (nrhs == 1 && n % 2 == 0)
    sym_gemv1_kernel<<<(unsigned)((n + 3) / 4), 256, 0, c.stream>>>(A, n, b, x);
  else
    sym_gemv_kernel<<<(unsigned)((n + 3) / 4), 256, 0, c.stream>>>(A, n, b, x, nrhs);
}

void imex_free(Ctx& c) {
  for (void* p : {(void*)c.d_imex_dofs, (void*)c.d_imex_s, (void*)c.d_imex_m,
                  (void*)c.d_imex_work, (void*)c.d_imex_flag})
    if (p) (void)hipFree(p);
  c.d_imex_dofs = nullptr;
  c.d_imex_s = c.d_imex_m = c.d_imex_work = nullptr;
  c.d_imex_flag = nullptr;
  c.imex_work_bytes = 0;
  c.imex_nc = -1;
  c.imex_dt = 0.0;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// x = A^{-1} b for nrhs right-hand sides of length n, A = L L^T given as the pair (L, L^T)
static fcw_status imex_solve(Ctx& c, const double* Lpair, int64_t n, int nrhs, const double* b,
                             double* x) {
  const size_t lds = (size_t)n * sizeof(double);
  // set once (not a stream operation)
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)chol_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      FCW_IMEX_MAX_NC * (int)sizeof(double));
  FCW_HIP(attr);
  chol_solve_kernel<<<nrhs, 256, lds, c.stream>>>(Lpair, Lpair + (size_t)n * n, n, b, x);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "IMEX triangular solves");
  return FCW_OK;
}

// Implicit set, dense S = M^cc + beta dt^2 K^cc and M^cc, their factors.
fcw_status imex_prepare(Ctx& c, double dt) {
  if (c.imex_nc >= 0 && c.imex_dt == dt) return FCW_OK;
  imex_free(c);
  int32_t *mark = nullptr, *pos = nullptr;
  auto fail = [&](fcw_status s) {
    if (mark) (void)hipFree(mark);
    if (pos) (void)hipFree(pos);
    imex_free(c);
    return s;
  };
  if (hipMalloc(&mark, c.nnodes * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&pos, c.nnodes * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c.d_imex_flag, sizeof(int32_t)) != hipSuccess) {
    set_error("IMEX: allocation of the node marks failed");
    return fail(FCW_E_NOMEM);
  }
  if (hipMemsetAsync(mark, 0, c.nnodes * sizeof(int32_t), c.stream) != hipSuccess)
    return fail(hip_fail(hipGetLastError(), "IMEX marks"));
  const int ns = c.n_s, nl = c.n_loc;
  if (c.n_cut_cand > 0)
    imex_mark_kernel<<<blocks_for(c.n_cut_cand * ns), 256, 0, c.stream>>>(
        c.d_info, c.d_cut_cells, c.n_cut_cand, c.dim, c.p, c.ncells[0], c.ncells[1], c.npts[0],
        c.npts[1], mark);
  int32_t ncn = 0;
  fcw_status st = exclusive_scan(c, mark, pos, c.nnodes, &ncn);
  if (st) return fail(st);
  const int64_t nc = (int64_t)ncn * c.ncomp;
  if (nc > FCW_IMEX_MAX_NC) {
    set_error("IMEX: %lld implicit DOFs exceed the dense limit %d", (long long)nc,
              FCW_IMEX_MAX_NC);
    return fail(FCW_E_UNSUPPORTED);
  }
  c.imex_ncn = ncn;
  if (nc > 0) {
    const size_t mat = (size_t)nc * nc * sizeof(double);
    if (hipMalloc(&c.d_imex_dofs, nc * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_s, 3 * mat) != hipSuccess ||
        hipMalloc(&c.d_imex_m, 3 * mat) != hipSuccess) {
      set_error("IMEX: allocation of the dense implicit matrices (%lld DOFs) failed",
                (long long)nc);
      return fail(FCW_E_NOMEM);
    }
    imex_dofs_kernel<<<blocks_for(c.nnodes), 256, 0, c.stream>>>(mark, pos, c.nnodes, ncn,
                                                                c.ncomp, c.d_imex_dofs);
    ImexAsm a{};
    a.dofs = c.d_imex_dofs;
    a.info = c.d_info;
    a.kref = c.d_kref;
    a.lref = c.d_lref;
    a.kcut = c.d_kcut;
    a.mcut = c.d_mcut;
    a.S = c.d_imex_s;
    a.M = c.d_imex_m;
    a.nc = nc;
    a.nnodes = c.nnodes;
    a.dim = c.dim;
    a.p = c.p;
    a.ns = ns;
    a.nl = nl;
    for (int k = 0; k < 3; ++k) {
      a.n[k] = c.ncells[k];
      a.np[k] = c.npts[k];
    }
    a.bdt2 = kBeta * dt * dt;
    const unsigned gy = (unsigned)std::min<int64_t>(nc, 65535);
    const unsigned gz = (unsigned)((nc + gy - 1) / gy);
    imex_assemble_kernel<<<dim3(blocks_for(nc), gy, gz), 256, 0, c.stream>>>(a);
    {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail(hip_fail(e, "IMEX assembly"));
    }
    if ((st = cholesky(c, c.d_imex_s, c.d_imex_s + (size_t)nc * nc, nc))) return fail(st);
    if ((st = cholesky(c, c.d_imex_m, c.d_imex_m + (size_t)nc * nc, nc))) return fail(st);
    // S^{-1} and (M^cc)^{-1}, column by column (symmetric: row r of the result is column r)
    for (double* f : {c.d_imex_s, c.d_imex_m}) {
      double* inv = f + 2 * (size_t)nc * nc;
      identity_kernel<<<blocks_for(nc * nc), 256, 0, c.stream>>>(inv, nc);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail(hip_fail(e, "IMEX identity"));
      if ((st = imex_solve(c, f, nc, (int)nc, inv, inv))) return fail(st);
    }
    {
      const hipError_t e = hipStreamSynchronize(c.stream);
      if (e != hipSuccess) return fail(hip_fail(e, "IMEX inverse"));
    }
  }
  (void)hipFree(mark);
  (void)hipFree(pos);
  c.imex_nc = nc;
  c.imex_dt = dt;
  return FCW_OK;
}

// nsteps IMEX steps; u, d [nrhs][ndof], v_c, a_c [nrhs][nc] (FP64, device)
fcw_status imex_run(Ctx& c, int nrhs, double* u, double* d, double* v_c, double* a_c,
                    double t0, double dt, int nsteps, int start, bool consistent) {
  const int64_t nc = c.imex_nc, ndof = c.ndof;
  const int64_t nv = nc * nrhs;
  // work: r (nrhs x ndof), then b, anew, uold, dold (nrhs x nc each), each part starting
  // on a 256-byte boundary
  auto up32 = [](size_t v) { return (v + 31) / 32 * 32; };
  const size_t nr = up32((size_t)nrhs * ndof), nvp = up32((size_t)nv);
  const size_t need = (nr + 4 * nvp) * sizeof(double);
  if (c.imex_work_bytes < need) {
    if (c.d_imex_work) FCW_HIP(hipFree(c.d_imex_work));
    c.d_imex_work = nullptr;
    c.imex_work_bytes = 0;
    FCW_HIP(hipMalloc(&c.d_imex_work, need));
    c.imex_work_bytes = need;
  }
  double* rk = c.d_imex_work;
  double* bv = rk + nr;
  double* an = bv + nvp;
  double* uold = an + nvp;
  const unsigned gb = blocks_for(nv);
  fcw_status st;
  if (consistent) {
    // central differences with the consistent cut-DOF mass (a = (M^cc)^{-1} (F - K u) on
    // the implicit DOFs, the diagonal elsewhere)
    double* dold = uold + nvp;
    for (int k = 0; k < nsteps; ++k) {
      const double t = t0 + k * dt;
      const int first = start && k == 0;
      if (nc > 0) {
        imex_gather_kernel<<<gb, 256, 0, c.stream>>>(u, c.d_imex_dofs, nc, ndof, nrhs, uold);
        imex_gather_kernel<<<gb, 256, 0, c.stream>>>(d, c.d_imex_dofs, nc, ndof, nrhs, dold);
        if ((st = launch_apply(c, nrhs, u, rk))) return st;
        imex_rhs_kernel<<<gb, 256, 0, c.stream>>>(rk, c.d_imex_dofs, c.d_src, nc, ndof, c.nnodes,
                                                  nrhs, c.dim, c.p, c.npts[0], c.npts[1], t, bv);
        solve_product(c, c.d_imex_m + 2 * (size_t)nc * nc, nc, bv, an, nrhs);
      }
      if ((st = run_steps(c, c.tile_choice, nrhs, u, d, c.d_ubuf, t, dt, 1, first))) return st;
      if (nc > 0)
        cons_fix_kernel<<<gb, 256, 0, c.stream>>>(u, d, c.d_imex_dofs, uold, dold, an, nc, ndof,
                                                  nrhs, (first ? 0.5 : 1.0) * dt * dt);
      FCW_HIP(hipGetLastError());
    }
    return FCW_OK;
  }
  if (start && nc > 0) {
    // a_0 from M^cc a_0 = F_0 - (K u_0) on the implicit DOFs
    if ((st = launch_apply(c, nrhs, u, rk))) return st;
    imex_rhs_kernel<<<gb, 256, 0, c.stream>>>(rk, c.d_imex_dofs, c.d_src, nc, ndof, c.nnodes, nrhs,
                                              c.dim, c.p, c.npts[0], c.npts[1], t0, bv);
    if ((st = imex_solve(c, c.d_imex_m, nc, nrhs, bv, a_c))) return st;
  }
  for (int k = 0; k < nsteps; ++k) {
    const double t = t0 + k * dt;
    if (nc > 0)
      imex_gather_kernel<<<gb, 256, 0, c.stream>>>(u, c.d_imex_dofs, nc, ndof, nrhs, uold);
    // explicit DOFs: one central-difference step of the explicit solver
    if ((st = run_steps(c, c.tile_choice, nrhs, u, d, c.d_ubuf, t, dt, 1, (start && k == 0))))
      return st;
    if (nc == 0) continue;
    imex_predict_kernel<<<gb, 256, 0, c.stream>>>(u, c.d_imex_dofs, uold, v_c, a_c, nc, ndof,
                                                  nrhs, dt);
    if ((st = launch_apply(c, nrhs, u, rk))) return st;
    imex_rhs_kernel<<<gb, 256, 0, c.stream>>>(rk, c.d_imex_dofs, c.d_src, nc, ndof, c.nnodes, nrhs,
                                              c.dim, c.p, c.npts[0], c.npts[1], t + dt, bv);
    solve_product(c, c.d_imex_s + 2 * (size_t)nc * nc, nc, bv, an, nrhs);
    imex_correct_kernel<<<gb, 256, 0, c.stream>>>(u, d, c.d_imex_dofs, uold, v_c, a_c, an, nc,
                                                  ndof, nrhs, dt);
    FCW_HIP(hipGetLastError());
  }
  return FCW_OK;
}

}  // namespace fcw
