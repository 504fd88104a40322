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
//      DOFs (left in a vector over the implicit DOFs by the previous step's corrector),
//      the explicit DOFs' new values serving as theirs;
//   3. b = F_{k+1} - K^c u_p on the implicit DOFs: the implicit rows of K (every column
//      they touch) assembled once as compressed sparse rows, 16 lanes per row;
//   4. S a_{k+1} = b, S = M^cc + beta dt^2 K^cc: a product with S^{-1}, formed once from
//      the Cholesky factor of S (forward and backward sweeps against the unit vectors,
//      one workgroup per column) and held as the 32 x 32 tiles of its upper triangle
//      (each off-diagonal tile serves its row block and, transposed, its column block);
//   5. v_{k+1} = v_k + dt ((1 - gamma) a_k + gamma a_{k+1}),
//      u_{k+1} = u_p + beta dt^2 a_{k+1} (in the kernel that sums the tile products).
//
// The same set-up serves central differences with the consistent cut-DOF mass (the
// consistent-mass spectral cell method, eq. cdm with M = diag(M^dd, M^cc)): per step
// a = (M^cc)^{-1} (F_k - K^c u_k) on the implicit DOFs, the lumped step elsewhere.
//
// The implicit set splits into blocks: implicit nodes linked through shared active
// cells (in a void field, the cut cells around one void or one cluster of voids).  S and
// M^cc have no entry between blocks, so each block is assembled dense (entry by entry
// from the cells around the two nodes, in a fixed order), factored on the device by a
// blocked right-looking Cholesky and inverted on its own.  The dense form bounds a block
// (FCW_IMEX_MAX_NC), not the whole set; one block that large (a percolating pore space)
// would need a sparse factorisation.
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

// node coordinates of a DOF
__device__ inline void dof_coords(const ImexAsm& a, int64_t g, int& comp, int x[3]) {
  comp = (int)(g / a.nnodes);
  const int64_t nd = g % a.nnodes;
  x[0] = (int)(nd % a.np[0]);
  x[1] = (int)((nd / a.np[0]) % a.np[1]);
  x[2] = (int)(nd / ((int64_t)a.np[0] * a.np[1]));
}

// K and M entries of the DOF pair (node xi, component ci), (node xj, component cj): the
// cells around node i, in a fixed order; those that also hold node j contribute
__device__ void pair_sums(const ImexAsm& a, const int xi[3], int ci, const int xj[3], int cj,
                          double& ks, double& ms) {
  ks = 0.0;
  ms = 0.0;
  for (int k = 0; k < a.dim; ++k)
    if (abs(xi[k] - xj[k]) > a.p) return;
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

__global__ void imex_assemble_kernel(ImexAsm a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
  if (i >= a.nc || j >= a.nc) return;
  int ci, cj, xi[3], xj[3];
  dof_coords(a, a.dofs[i], ci, xi);
  dof_coords(a, a.dofs[j], cj, xj);
  double ks, ms;
  pair_sums(a, xi, ci, xj, cj, ks, ms);
  a.M[i * a.nc + j] = ms;
  a.S[i * a.nc + j] = ms + a.bdt2 * ks;
}

// The implicit rows of K, padded to W = ncomp (2p+1)^dim slots: slot (cj, o) of row i is
// the DOF of component cj at node x_i + o, o in [-p, p]^dim (x fastest).  The column is
// that DOF's global index, or -(its implicit index + 1) when it is implicit (the steps
// take those values from a vector over the implicit DOFs).  A slot off the grid holds row
// i's own column with the value 0.
__global__ void imex_kc_assemble_kernel(ImexAsm a, int W, const int32_t* mark,
                                        const int32_t* pos, int64_t ncn, int32_t* col,
                                        double* val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nc * W) return;
  const int64_t i = t / W;
  int w = (int)(t % W);
  const int64_t gi = a.dofs[i];
  int ci, xi[3];
  dof_coords(a, gi, ci, xi);
  const int side = 2 * a.p + 1;
  int span = 1;
  for (int k = 0; k < a.dim; ++k) span *= side;
  const int cj = w / span;
  w %= span;
  int xj[3] = {0, 0, 0};
  bool in = true;
  for (int k = 0; k < a.dim; ++k) {
    xj[k] = xi[k] + (w % side) - a.p;
    w /= side;
    if (xj[k] < 0 || xj[k] >= a.np[k]) in = false;
  }
  double ks = 0.0, ms;
  int cc = ci;
  int64_t nj = gi % a.nnodes;
  if (in) {
    pair_sums(a, xi, ci, xj, cj, ks, ms);
    cc = cj;
    nj = xj[0] + (int64_t)a.np[0] * (xj[1] + (int64_t)a.np[1] * xj[2]);
  }
  col[t] = mark[nj] ? (int32_t)(-(cc * ncn + pos[nj]) - 1) : (int32_t)(cc * a.nnodes + nj);
  val[t] = ks;
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

// ---- the inverses as the 32 x 32 tiles of their upper triangle ----

constexpr int kTile = 32;

// packed position of tile (I, J), I <= J, in a T x T tile grid (row I's tiles follow
// those of rows 0 .. I-1)
__host__ __device__ inline int64_t tile_index(int64_t I, int64_t J, int64_t T) {
  return I * T - I * (I - 1) / 2 + (J - I);
}

// tile (I, J) at packed position q
__device__ inline void tile_at(int64_t q, int64_t T, int64_t& I, int64_t& J) {
  const double b = 2.0 * (double)T + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)q)) * 0.5);
  i = max((int64_t)0, min(i, T - 1));
  while (i > 0 && tile_index(i, i, T) > q) --i;
  while (i + 1 < T && tile_index(i + 1, i + 1, T) <= q) ++i;
  I = i;
  J = i + (q - tile_index(i, i, T));
}

// P[tile (I, J)][r][c] = (A_ij + A_ji) / 2 at i = 32 I + r, j = 32 J + c (0 beyond n),
// for the T (T + 1) / 2 upper tiles of one block in packed order, and the tiles'
// descriptors: the inverse from column-wise solves is symmetric up to rounding; both
// halves are kept
// one packed tile: (I, J) in its block of n DOFs and T tile rows, the block's first
// block-order position and the offset of its partial products (per right-hand side)
struct TileDesc {
  int32_t I, J, n, T;
  int64_t moff, poff;
};

__global__ void pack_inverse_tiles_kernel(const double* A, int64_t n, int64_t T, double* P,
                                          TileDesc* tiles, int64_t moff, int64_t poff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T * (T + 1) / 2 * kTile * kTile) return;
  const int64_t q = t / (kTile * kTile);
  const int e = (int)(t % (kTile * kTile));
  int64_t I, J;
  tile_at(q, T, I, J);
  const int64_t i = I * kTile + e / kTile, j = J * kTile + e % kTile;
  P[t] = (i < n && j < n) ? 0.5 * (A[i * n + j] + A[j * n + i]) : 0.0;
  if (tiles && e == 0) tiles[q] = TileDesc{(int32_t)I, (int32_t)J, (int32_t)n, (int32_t)T, moff, poff};
}

// one block of the implicit set: its n DOFs sit at block-order positions moff .. moff+n-1,
// its T = ceil(n / 32) tile rows' partial products at part + nrhs * poff
struct ImexBlock {
  int64_t moff, poff;
  int32_t n, T;
};

// Partial products of x = A b over the packed upper tiles of the blocks: the rows of tile
// (I, J) of a block against b's block J go to part[J][r][block I] and, for I < J, its
// columns against b's block I to part[I][r][block J], where part is the block's
// [T][nrhs][32 T] array; every entry is written by exactly one tile, and x_i is the sum of
// part[0 .. T-1][r][i].  b and x are in block order ([nrhs][nc]).
// One wave takes TPW consecutive tiles and issues all their loads before the first
// product.  Lane layout: columns 2 cp, 2 cp + 1 (cp = lane mod 16), rows rs + 4 k (k < 8,
// rs = lane / 16): each load instruction reads four 256-byte tile rows.
struct TileIn {
  double2 v[8];
  double bI, bJ;  // b at rows 32 I + (lane mod 32) and 32 J + (lane mod 32), first rhs
};

__device__ inline void tile_load(const double* P, const TileDesc& td, int64_t q,
                                 const double* b, int lane, TileIn& in) {
  const int cp = lane & 15, rs = lane >> 4;
  const int64_t iB = (int64_t)td.I * kTile + (lane & 31), jB = (int64_t)td.J * kTile + (lane & 31);
  in.bI = iB < td.n ? b[td.moff + iB] : 0.0;
  in.bJ = jB < td.n ? b[td.moff + jB] : 0.0;
  // the tiles are read once per product: nontemporal loads keep them from displacing the
  // vectors and partial products in the caches
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v* tile = (const d2v*)(P + q * kTile * kTile);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const d2v x = __builtin_nontemporal_load(tile + (rs + 4 * k) * (kTile / 2) + cp);
    in.v[k] = make_double2(x.x, x.y);
  }
}

__device__ inline void tile_products(const TileDesc& td, const TileIn& in, const double* b,
                                     int64_t nc, int nrhs, double* part, int lane) {
  const int cp = lane & 15, rs = lane >> 4;
  const int64_t I = td.I, J = td.J, n = td.n;
  const int64_t stride = (int64_t)td.T * kTile;
  double* pb = part + nrhs * td.poff;
  const bool off_diag = I < J;
  const int64_t iB = I * kTile + (lane & 31), jB = J * kTile + (lane & 31);
  const int b3 = (cp >> 3) & 1, b2 = (cp >> 2) & 1, b1 = (cp >> 1) & 1;
  for (int r = 0; r < nrhs; ++r) {
    double bI = in.bI, bJ = in.bJ;
    if (r > 0) {
      const double* br = b + (int64_t)r * nc + td.moff;
      bI = iB < n ? br[iB] : 0.0;
      bJ = jB < n ? br[jB] : 0.0;
    }
    const double bj0 = __shfl(bJ, 2 * cp), bj1 = __shfl(bJ, 2 * cp + 1);
    double s[8];
    double cs0 = 0.0, cs1 = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k] = in.v[k].x * bj0 + in.v[k].y * bj1;
      const double bi = __shfl(bI, rs + 4 * k);
      cs0 += in.v[k].x * bi;
      cs1 += in.v[k].y * bi;
    }
    // row sums over the 16 lanes of a row group: three halving exchanges leave each lane
    // one row (k = 4 b3 + 2 b2 + b1), then one butterfly step
    double t4[4], t2[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double send = b3 ? s[j] : s[j + 4];
      const double keep = b3 ? s[j + 4] : s[j];
      t4[j] = keep + __shfl_xor(send, 8);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double send = b2 ? t4[j] : t4[j + 2];
      const double keep = b2 ? t4[j + 2] : t4[j];
      t2[j] = keep + __shfl_xor(send, 4);
    }
    double w;
    {
      const double send = b1 ? t2[0] : t2[1];
      const double keep = b1 ? t2[1] : t2[0];
      w = keep + __shfl_xor(send, 2);
    }
    w += __shfl_xor(w, 1);
    if ((cp & 1) == 0)
      pb[(J * nrhs + r) * stride + I * kTile + rs + 4 * (4 * b3 + 2 * b2 + b1)] = w;
    if (off_diag) {
      // column sums over the four row groups
      cs0 += __shfl_xor(cs0, 16);
      cs1 += __shfl_xor(cs1, 16);
      cs0 += __shfl_xor(cs0, 32);
      cs1 += __shfl_xor(cs1, 32);
      if (lane < 16)
        *(double2*)(pb + (I * nrhs + r) * stride + J * kTile + 2 * cp) = make_double2(cs0, cs1);
    }
  }
}

template <int TPW>
__global__ __launch_bounds__(256) void symp_tile_kernel(const double* P, const TileDesc* tiles,
                                                        int64_t ntiles, const double* b,
                                                        int64_t nc, int nrhs, double* part) {
  const int lane = threadIdx.x & 63;
  // wave-uniform tile index: the descriptors come through the scalar unit
  const int64_t q0 =
      TPW * ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
  if (q0 >= ntiles) return;
  TileDesc td[TPW];
  TileIn in[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    td[j] = tiles[min(q0 + j, ntiles - 1)];
    if (q0 + j < ntiles) tile_load(P, td[j], q0 + j, b, lane, in[j]);
  }
#pragma unroll
  for (int j = 0; j < TPW; ++j)
    if (q0 + j < ntiles) tile_products(td[j], in[j], b, nc, nrhs, part, lane);
}

// tiles per wave of symp_tile_kernel
constexpr int kTilesPerWave = 1;

typedef double symp_f64x4 __attribute__((ext_vector_type(4)));

// The same tile products for several right-hand sides on the FP64 matrix cores, 16
// right-hand sides per pass: the wave's tile goes to LDS (rows padded to 33 doubles), then
// Y = A B_J (32 x 16, B_J the right-hand sides' block J) and, for I < J, Z = A^T B_I, each
// as two 16-row halves of eight k-steps of v_mfma_f64_16x16x4f64.  Operands: lane
// l16 + 16 k4 holds A[l16][k4] and B[k4][l16]; the result lane holds rows 4 v + k4
// (v < 4) of column l16.
__global__ __launch_bounds__(256) void symp_tile_mfma_kernel(const double* P,
                                                             const TileDesc* tiles,
                                                             int64_t ntiles, const double* b,
                                                             int64_t nc, int nrhs,
                                                             double* part) {
  constexpr int LD = kTile + 1;
  __shared__ double lds[4][kTile * LD];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  if (q >= ntiles) return;
  const TileDesc td = tiles[q];
  double* A = lds[wave];
  {
    const int cp = lane & 15, rs = lane >> 4;
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v* tile = (const d2v*)(P + q * kTile * kTile);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const d2v x = __builtin_nontemporal_load(tile + (rs + 4 * k) * (kTile / 2) + cp);
      A[(rs + 4 * k) * LD + 2 * cp] = x.x;
      A[(rs + 4 * k) * LD + 2 * cp + 1] = x.y;
    }
  }
  // LDS accesses of one wave complete in order; the barrier keeps the compiler's order
  __builtin_amdgcn_wave_barrier();
  const int l16 = lane & 15, k4 = lane >> 4;
  const int64_t I = td.I, J = td.J, n = td.n;
  const int64_t stride = (int64_t)td.T * kTile;
  double* pb = part + nrhs * td.poff;
  const bool off_diag = I < J;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int rr = r0 + l16;
    const bool rv = rr < nrhs;
    const double* br = b + (int64_t)(rv ? rr : 0) * nc + td.moff;
    symp_f64x4 y0 = {0.0, 0.0, 0.0, 0.0}, y1 = y0, z0 = y0, z1 = y0;
#pragma unroll
    for (int ks = 0; ks < kTile / 4; ++ks) {
      const int k = 4 * ks + k4;
      const int64_t jk = J * kTile + k, ik = I * kTile + k;
      const double bJ = (rv && jk < n) ? br[jk] : 0.0;
      y0 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[l16 * LD + k], bJ, y0, 0, 0, 0);
      y1 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(16 + l16) * LD + k], bJ, y1, 0, 0, 0);
      if (off_diag) {
        const double bI = (rv && ik < n) ? br[ik] : 0.0;
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k * LD + l16], bI, z0, 0, 0, 0);
        z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k * LD + 16 + l16], bI, z1, 0, 0, 0);
      }
    }
    if (r0 + 16 >= nrhs) {
      // last pass: the tile is no longer needed, so its LDS takes the results (Y in rows
      // 0..15, Z in rows 16..31, one row of 32 positions per right-hand side), written out
      // as whole 256-byte rows
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + k4;
        A[l16 * LD + i] = y0[v];
        A[l16 * LD + 16 + i] = y1[v];
        A[(16 + l16) * LD + i] = z0[v];
        A[(16 + l16) * LD + 16 + i] = z1[v];
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int rl = t * 2 + (lane >> 5), pos = lane & 31;
        if (r0 + rl < nrhs) {
          pb[(J * nrhs + r0 + rl) * stride + I * kTile + pos] = A[rl * LD + pos];
          if (off_diag) pb[(I * nrhs + r0 + rl) * stride + J * kTile + pos] = A[(16 + rl) * LD + pos];
        }
      }
    } else {
      double* py = pb + (J * nrhs + rr) * stride + I * kTile;
      double* pz = pb + (I * nrhs + rr) * stride + J * kTile;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + k4;
        py[i] = y0[v];
        py[16 + i] = y1[v];
        if (off_diag) {
          pz[i] = z0[v];
          pz[16 + i] = z1[v];
        }
      }
    }
  }
}

// the updates that consume x = A b on the implicit DOFs ([nrhs][nc] vectors)
struct ImexUpd {
  double* u;             // [nrhs][ndof]
  double* d;             // [nrhs][ndof]
  const int64_t* dofs;   // [nc]
  double* uold;          // u_k; receives u_{k+1}
  double* dold;          // d_k; receives d_{k+1} (consistent mass)
  double* v;             // v_k -> v_{k+1} (IMEX)
  double* a;             // a_k -> a_{k+1} (IMEX)
  double* upred;         // IMEX predictor of this step; receives the next step's
  int64_t ndof;
  double dt;             // IMEX step
  double w;              // consistent mass: dt^2, or dt^2 / 2 on a starting step
};

// IMEX corrector with a_{k+1} = x: v += dt ((1 - gamma) a_k + gamma a_{k+1}),
// u = u_p + beta dt^2 a_{k+1}, d = u - u_k; u_{k+1} and the next step's predictor kept
__device__ inline void imex_correct_at(const ImexUpd& e, int64_t t, int64_t r, int64_t i,
                                       double an) {
  const int64_t g = r * e.ndof + e.dofs[i];
  const double vn = e.v[t] + e.dt * ((1.0 - kGamma) * e.a[t] + kGamma * an);
  const double un = e.upred[t] + kBeta * e.dt * e.dt * an;
  e.v[t] = vn;
  e.u[g] = un;
  e.d[g] = un - e.uold[t];
  e.uold[t] = un;
  e.a[t] = an;
  e.upred[t] = un + e.dt * vn + (0.5 - kBeta) * e.dt * e.dt * an;
}

// consistent-mass central differences with a = x: d = d_k + w a, u = u_k + d
__device__ inline void cons_fix_at(const ImexUpd& e, int64_t t, int64_t r, int64_t i,
                                   double an) {
  const int64_t g = r * e.ndof + e.dofs[i];
  const double dn = e.dold[t] + e.w * an;
  const double un = e.uold[t] + dn;
  e.d[g] = dn;
  e.u[g] = un;
  e.dold[t] = dn;
  e.uold[t] = un;
}

constexpr int kUpdStore = 0, kUpdImex = 1, kUpdCons = 2;

// x at block-order position m: the sum over Y of its block's part[Y][r][m - moff], handed
// to the update MODE at the implicit DOF members[m] (kUpdStore: a = x).  16 positions per
// workgroup, sixteen groups of lanes each summing every sixteenth Y, then the groups in a
// fixed order.
template <int MODE>
__global__ __launch_bounds__(256) void symp_reduce_kernel(const double* part,
                                                          const int32_t* pblk,
                                                          const int32_t* members,
                                                          const ImexBlock* blocks, int64_t nc,
                                                          int nrhs, ImexUpd e) {
  __shared__ double red[16][16];
  const int il = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t nb = (nc + 15) / 16;
  const int64_t r = blockIdx.x / nb;
  const int64_t m = (blockIdx.x % nb) * 16 + il;
  double s = 0.0;
  if (m < nc) {
    const ImexBlock bk = blocks[pblk[m]];
    const int64_t stride = (int64_t)bk.T * kTile;
    const double* p = part + nrhs * bk.poff + r * stride + (m - bk.moff);
    const int64_t ys = nrhs * stride;
    int64_t y = g;
    // four loads in flight, summed in the order of y
    for (; y + 48 < bk.T; y += 64) {
      const double a0 = p[y * ys], a1 = p[(y + 16) * ys], a2 = p[(y + 32) * ys],
                   a3 = p[(y + 48) * ys];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; y < bk.T; y += 16) s += p[y * ys];
  }
  red[g][il] = s;
  __syncthreads();
  if (g == 0 && m < nc) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += red[q][il];
    const int64_t i = members[m], t = r * nc + i;
    if (MODE == kUpdStore)
      e.a[t] = acc;
    else if (MODE == kUpdImex)
      imex_correct_at(e, t, r, i, acc);
    else
      cons_fix_at(e, t, r, i, acc);
  }
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

// the predictor u_p = u_k + dt v + (1/2 - beta) dt^2 a on the implicit DOFs
__global__ void imex_predict_kernel(const double* uold, const double* v, const double* a,
                                    int64_t nv, double dt, double* upred) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nv) return;
  upred[t] = uold[t] + dt * v[t] + (0.5 - kBeta) * dt * dt * a[t];
}

// F(t) of right-hand side r at DOF g (the point source of the call, 0 without one)
__device__ inline double source_at(const SourceDev* src, int64_t r, int64_t g, int64_t nnodes,
                                   int dim, int p, int np0, int np1, double t) {
  if (!src) return 0.0;
  const SourceDev& s = src[r];
  const int comp = (int)(g / nnodes);
  const int64_t node = g % nnodes;
  const int x = (int)(node % np0), y = (int)((node / np0) % np1),
            z = (int)(node / ((int64_t)np0 * np1));
  const int sx = x - s.cell[0] * p, sy = y - s.cell[1] * p, sz = (dim == 3) ? z - s.cell[2] * p : 0;
  const int np1p = p + 1;
  const int ns = (dim == 3) ? np1p * np1p * np1p : np1p * np1p;
  if (sx >= 0 && sx <= p && sy >= 0 && sy <= p && sz >= 0 && sz <= p)
    return ricker(t, s.f0) * s.b[comp * ns + sx + np1p * (sy + np1p * sz)];
  return 0.0;
}

// nonzero slots of each padded row
__global__ void imex_kc_count_kernel(const double* val, int W, int64_t nc, int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int32_t k = 0;
  for (int w = 0; w < W; ++w) k += val[i * W + w] != 0.0;
  cnt[i] = k;
}

// the padded rows' nonzero slots, in slot order, at ptr[i] .. ptr[i+1]-1
__global__ void imex_kc_compact_kernel(const int32_t* ecol, const double* eval, int W,
                                       int64_t nc, const int32_t* ptr, int32_t* col,
                                       double* val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int64_t o = ptr[i];
  for (int w = 0; w < W; ++w) {
    const double v = eval[i * W + w];
    if (v != 0.0) {
      col[o] = ecol[i * W + w];
      val[o] = v;
      ++o;
    }
  }
}

// b = F(t) - K^c u on the implicit DOFs (written in block order: b[r][cpos[i]]), u from
// uimp [nrhs][nc] on the implicit DOFs and from u [nrhs][ndof] elsewhere: one wave per
// 16 lanes per implicit row of the compressed sparse rows, four rows per wave (lanes over
// the row's entries, a fixed butterfly for the sum)
__global__ __launch_bounds__(256) void imex_kc_rhs_kernel(
    const int32_t* ptr, const int32_t* col, const double* val, const double* u, const double* uimp,
    const int64_t* dofs, const SourceDev* src, int64_t nc, int64_t ndof, int64_t nnodes,
    int nrhs, int dim, int p, int np0, int np1, double t, const int32_t* cpos, double* b) {
  const int lane = threadIdx.x & 15;
  const int64_t i = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  // rows past the end still take part in the shuffles (empty entry range)
  const int32_t k0 = i < nc ? ptr[i] : 0, k1 = i < nc ? ptr[i + 1] : 0;
  for (int r = 0; r < nrhs; ++r) {
    const double* ur = u + (int64_t)r * ndof;
    const double* ui = uimp + (int64_t)r * nc;
    double s = 0.0;
    for (int32_t k = k0 + lane; k < k1; k += 16) {
      const int32_t cw = col[k];
      s += val[k] * (cw >= 0 ? ur[cw] : ui[-cw - 1]);
    }
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && i < nc)
      b[(int64_t)r * nc + cpos[i]] = source_at(src, r, dofs[i], nnodes, dim, p, np0, np1, t) - s;
  }
}

// part = the tile products of x = A b (A the packed upper tiles of the blocks of the
// inverse of S or M^cc; b in block order)
static void symp_tiles(Ctx& c, const double* A, const double* b, int nrhs, double* part) {
  if (nrhs >= 2) {  // several right-hand sides: the matrix cores
    symp_tile_mfma_kernel<<<(unsigned)((c.imex_ntiles + 3) / 4), 256, 0, c.stream>>>(
        A, (const TileDesc*)c.d_imex_tiles, c.imex_ntiles, b, c.imex_nc, nrhs, part);
    return;
  }
  constexpr int per_block = 4 * kTilesPerWave;
  symp_tile_kernel<kTilesPerWave>
      <<<(unsigned)((c.imex_ntiles + per_block - 1) / per_block), 256, 0, c.stream>>>(
          A, (const TileDesc*)c.d_imex_tiles, c.imex_ntiles, b, c.imex_nc, nrhs, part);
}

// the reduction of the tile products, fused with the update that consumes x
template <int MODE>
static void symp_finish(Ctx& c, const double* part, int nrhs, const ImexUpd& e) {
  const int64_t n = c.imex_nc;
  symp_reduce_kernel<MODE><<<(unsigned)(((n + 15) / 16) * nrhs), 256, 0, c.stream>>>(
      part, c.d_imex_pblk, c.d_imex_members, (const ImexBlock*)c.d_imex_blocks, n, nrhs, e);
}

void imex_free(Ctx& c) {
  for (void* p : {(void*)c.d_imex_dofs, (void*)c.d_imex_s, (void*)c.d_imex_m,
                  (void*)c.d_imex_sp, (void*)c.d_imex_mp, (void*)c.d_imex_kcol,
                  (void*)c.d_imex_kval, (void*)c.d_imex_work, (void*)c.d_imex_flag,
                  (void*)c.d_imex_cpos, (void*)c.d_imex_members, (void*)c.d_imex_pblk,
                  (void*)c.d_imex_kptr, c.d_imex_blocks, c.d_imex_tiles})
    if (p) (void)hipFree(p);
  c.d_imex_dofs = nullptr;
  c.d_imex_s = c.d_imex_m = c.d_imex_sp = c.d_imex_mp = c.d_imex_work = nullptr;
  c.d_imex_kcol = c.d_imex_kptr = c.d_imex_cpos = c.d_imex_members = c.d_imex_pblk = nullptr;
  c.d_imex_kval = nullptr;
  c.d_imex_blocks = c.d_imex_tiles = nullptr;
  c.imex_nblk = 0;
  c.imex_largest = c.imex_ntiles = c.imex_part = 0;
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
  if (c.ndof > INT32_MAX) {
    set_error("IMEX: %lld DOFs exceed the 32-bit column indices", (long long)c.ndof);
    return fail(FCW_E_UNSUPPORTED);
  }
  c.imex_ncn = ncn;
  if (nc > 0) {
    // Blocks of the implicit set: implicit nodes are linked when they share an active cell
    // (S and M^cc have no entry between DOFs of different blocks).  Union-find on the host
    // over the cells; blocks are numbered by their lowest node, their DOFs ordered
    // component-major, then by node.
    const int64_t ncells = (int64_t)c.ncells[0] * c.ncells[1] * (c.dim == 3 ? c.ncells[2] : 1);
    std::vector<int32_t> h_mark(c.nnodes), h_pos(c.nnodes), h_info(ncells);
    if (hipMemcpyAsync(h_mark.data(), mark, c.nnodes * sizeof(int32_t), hipMemcpyDeviceToHost,
                       c.stream) != hipSuccess ||
        hipMemcpyAsync(h_pos.data(), pos, c.nnodes * sizeof(int32_t), hipMemcpyDeviceToHost,
                       c.stream) != hipSuccess ||
        hipMemcpyAsync(h_info.data(), c.d_info, ncells * sizeof(int32_t),
                       hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
      return fail(hip_fail(hipGetLastError(), "IMEX node marks to the host"));
    std::vector<int64_t> node_of(ncn);
    for (int64_t nd = 0; nd < c.nnodes; ++nd)
      if (h_mark[nd]) node_of[h_pos[nd]] = nd;
    std::vector<int32_t> par(ncn);
    for (int32_t j = 0; j < ncn; ++j) par[j] = j;
    auto find = [&](int32_t x) {
      while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
      }
      return x;
    };
    const int P1 = c.p + 1, nz = (c.dim == 3) ? P1 : 1;
    for (int64_t cell = 0; cell < ncells; ++cell) {
      if (h_info[cell] == kInfoOut) continue;
      const int64_t cx = cell % c.ncells[0], cy = (cell / c.ncells[0]) % c.ncells[1],
                    cz = cell / ((int64_t)c.ncells[0] * c.ncells[1]);
      int32_t first = -1;
      for (int k2 = 0; k2 < nz; ++k2)
        for (int k1 = 0; k1 < P1; ++k1)
          for (int k0 = 0; k0 < P1; ++k0) {
            const int64_t nd = (cx * c.p + k0) +
                               (int64_t)c.npts[0] * ((cy * c.p + k1) +
                                                     (int64_t)c.npts[1] * (cz * c.p + k2));
            if (!h_mark[nd]) continue;
            const int32_t j = h_pos[nd];
            if (first < 0) {
              first = j;
              continue;
            }
            const int32_t ra = find(first), rb = find(j);
            if (ra != rb) par[std::max(ra, rb)] = std::min(ra, rb);
          }
    }
    std::vector<int32_t> lab(ncn), rank(ncn), root_lab(ncn, -1), cnt;
    for (int32_t j = 0; j < ncn; ++j) {
      const int32_t rt = find(j);
      if (root_lab[rt] < 0) {
        root_lab[rt] = (int32_t)cnt.size();
        cnt.push_back(0);
      }
      lab[j] = root_lab[rt];
      rank[j] = cnt[lab[j]]++;
    }
    const int32_t nblk = (int32_t)cnt.size();
    std::vector<ImexBlock> blk(nblk);
    std::vector<int64_t> toff(nblk);
    int64_t moff = 0, poff = 0, ntiles = 0, nmax = 0;
    for (int32_t q = 0; q < nblk; ++q) {
      const int64_t n = (int64_t)cnt[q] * c.ncomp, T = (n + kTile - 1) / kTile;
      if (n > FCW_IMEX_MAX_NC) {
        set_error("IMEX: a block of %lld coupled implicit DOFs exceeds the dense limit %d",
                  (long long)n, FCW_IMEX_MAX_NC);
        return fail(FCW_E_UNSUPPORTED);
      }
      blk[q] = ImexBlock{moff, poff, (int32_t)n, (int32_t)T};
      toff[q] = ntiles;
      moff += n;
      poff += T * T * kTile;
      ntiles += T * (T + 1) / 2;
      nmax = std::max(nmax, n);
    }
    std::vector<int32_t> h_cpos(nc), h_members(nc), h_pblk(nc);
    std::vector<int64_t> h_cdofs(nc);
    for (int k = 0; k < c.ncomp; ++k)
      for (int32_t j = 0; j < ncn; ++j) {
        const ImexBlock& bk = blk[lab[j]];
        const int64_t i = (int64_t)k * ncn + j;
        const int64_t m = bk.moff + (int64_t)k * cnt[lab[j]] + rank[j];
        h_cpos[i] = (int32_t)m;
        h_members[m] = (int32_t)i;
        h_pblk[m] = lab[j];
        h_cdofs[m] = (int64_t)k * c.nnodes + node_of[j];
      }
    c.imex_nblk = nblk;
    c.imex_largest = nmax;
    c.imex_ntiles = ntiles;
    c.imex_part = poff;
    int W = c.ncomp;
    for (int k = 0; k < c.dim; ++k) W *= 2 * c.p + 1;
    if (nc * W > INT32_MAX) {
      set_error("IMEX: %lld implicit DOFs x %d stencil slots exceed 32-bit row offsets",
                (long long)nc, W);
      return fail(FCW_E_UNSUPPORTED);
    }
    int64_t* d_cdofs = nullptr;
    int32_t *ecol = nullptr, *kcnt = nullptr;
    double* eval = nullptr;
    const size_t mat = (size_t)nmax * nmax * sizeof(double);
    const size_t packed = (size_t)ntiles * kTile * kTile * sizeof(double);
    auto fail2 = [&](fcw_status st2) {
      for (void* p : {(void*)d_cdofs, (void*)ecol, (void*)eval, (void*)kcnt})
        if (p) (void)hipFree(p);
      return fail(st2);
    };
    if (hipMalloc(&c.d_imex_dofs, nc * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&d_cdofs, nc * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_cpos, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_members, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_pblk, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_blocks, nblk * sizeof(ImexBlock)) != hipSuccess ||
        hipMalloc(&c.d_imex_tiles, ntiles * sizeof(TileDesc)) != hipSuccess ||
        hipMalloc(&c.d_imex_s, 3 * mat) != hipSuccess ||
        hipMalloc(&c.d_imex_m, 3 * mat) != hipSuccess ||
        hipMalloc(&c.d_imex_sp, packed) != hipSuccess ||
        hipMalloc(&c.d_imex_mp, packed) != hipSuccess ||
        hipMalloc(&c.d_imex_kptr, (nc + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&kcnt, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&ecol, (size_t)nc * W * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&eval, (size_t)nc * W * sizeof(double)) != hipSuccess) {
      set_error("IMEX: allocation of the implicit matrices (%lld DOFs, largest block %lld) "
                "failed", (long long)nc, (long long)nmax);
      return fail2(FCW_E_NOMEM);
    }
    if (hipMemcpyAsync(d_cdofs, h_cdofs.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice,
                       c.stream) != hipSuccess ||
        hipMemcpyAsync(c.d_imex_cpos, h_cpos.data(), nc * sizeof(int32_t),
                       hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipMemcpyAsync(c.d_imex_members, h_members.data(), nc * sizeof(int32_t),
                       hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipMemcpyAsync(c.d_imex_pblk, h_pblk.data(), nc * sizeof(int32_t),
                       hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipMemcpyAsync(c.d_imex_blocks, blk.data(), nblk * sizeof(ImexBlock),
                       hipMemcpyHostToDevice, c.stream) != hipSuccess)
      return fail2(hip_fail(hipGetLastError(), "IMEX block tables"));
    imex_dofs_kernel<<<blocks_for(c.nnodes), 256, 0, c.stream>>>(mark, pos, c.nnodes, ncn,
                                                                c.ncomp, c.d_imex_dofs);
    ImexAsm a{};
    a.info = c.d_info;
    a.kref = c.d_kref;
    a.lref = c.d_lref;
    a.kcut = c.d_kcut;
    a.mcut = c.d_mcut;
    a.S = c.d_imex_s;
    a.M = c.d_imex_m;
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
    // per block: dense S and M^cc, Cholesky, inverses, packed upper tiles
    for (int32_t q = 0; q < nblk; ++q) {
      const int64_t n = blk[q].n, T = blk[q].T;
      a.dofs = d_cdofs + blk[q].moff;
      a.nc = n;
      const unsigned gy = (unsigned)std::min<int64_t>(n, 65535);
      const unsigned gz = (unsigned)((n + gy - 1) / gy);
      imex_assemble_kernel<<<dim3(blocks_for(n), gy, gz), 256, 0, c.stream>>>(a);
      {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail2(hip_fail(e, "IMEX assembly"));
      }
      if ((st = cholesky(c, c.d_imex_s, c.d_imex_s + (size_t)n * n, n))) return fail2(st);
      if ((st = cholesky(c, c.d_imex_m, c.d_imex_m + (size_t)n * n, n))) return fail2(st);
      // S^{-1} and (M^cc)^{-1}, column by column
      for (double* fm : {c.d_imex_s, c.d_imex_m}) {
        double* inv = fm + 2 * (size_t)n * n;
        identity_kernel<<<blocks_for(n * n), 256, 0, c.stream>>>(inv, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail2(hip_fail(e, "IMEX identity"));
        if ((st = imex_solve(c, fm, n, (int)n, inv, inv))) return fail2(st);
      }
      const int64_t np = T * (T + 1) / 2 * kTile * kTile;
      const size_t off = (size_t)toff[q] * kTile * kTile;
      pack_inverse_tiles_kernel<<<blocks_for(np), 256, 0, c.stream>>>(
          c.d_imex_s + 2 * (size_t)n * n, n, T, c.d_imex_sp + off,
          (TileDesc*)c.d_imex_tiles + toff[q], blk[q].moff, blk[q].poff);
      pack_inverse_tiles_kernel<<<blocks_for(np), 256, 0, c.stream>>>(
          c.d_imex_m + 2 * (size_t)n * n, n, T, c.d_imex_mp + off, nullptr, 0, 0);
      {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail2(hip_fail(e, "IMEX packing"));
      }
    }
    // the implicit rows of K (rows in implicit order): padded, then compressed to their
    // nonzero entries
    a.dofs = c.d_imex_dofs;
    a.nc = nc;
    imex_kc_assemble_kernel<<<blocks_for(nc * W), 256, 0, c.stream>>>(a, W, mark, pos, ncn,
                                                                      ecol, eval);
    imex_kc_count_kernel<<<blocks_for(nc), 256, 0, c.stream>>>(eval, W, nc, kcnt);
    {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail2(hip_fail(e, "IMEX stiffness rows"));
    }
    int32_t nnz = 0;
    if ((st = exclusive_scan(c, kcnt, c.d_imex_kptr, nc, &nnz))) return fail2(st);
    if (hipMemcpyAsync(c.d_imex_kptr + nc, &nnz, sizeof(int32_t), hipMemcpyHostToDevice,
                       c.stream) != hipSuccess ||
        hipMalloc(&c.d_imex_kcol, std::max<int64_t>(nnz, 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c.d_imex_kval, std::max<int64_t>(nnz, 1) * sizeof(double)) != hipSuccess) {
      set_error("IMEX: allocation of the implicit rows of K (%d entries) failed", nnz);
      return fail2(FCW_E_NOMEM);
    }
    imex_kc_compact_kernel<<<blocks_for(nc), 256, 0, c.stream>>>(
        ecol, eval, W, nc, c.d_imex_kptr, c.d_imex_kcol, c.d_imex_kval);
    {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail2(hip_fail(e, "IMEX stiffness rows"));
    }
    {
      const hipError_t e = hipStreamSynchronize(c.stream);
      if (e != hipSuccess) return fail2(hip_fail(e, "IMEX set-up"));
    }
    // the dense blocks, their factors and inverses are not used by the steps
    (void)hipFree(d_cdofs);
    (void)hipFree(ecol);
    (void)hipFree(eval);
    (void)hipFree(kcnt);
    (void)hipFree(c.d_imex_s);
    (void)hipFree(c.d_imex_m);
    c.d_imex_s = c.d_imex_m = nullptr;
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
  // work: b, u_k, d_k and the predictor on the implicit DOFs (nrhs x nc each), then the
  // tile products of the inverse (per block [T][nrhs][32 T]), each part on a 256-byte
  // boundary
  auto up32 = [](size_t v) { return (v + 31) / 32 * 32; };
  const size_t nvp = up32((size_t)nv), npart = (size_t)nrhs * c.imex_part;
  const size_t need = (4 * nvp + npart) * sizeof(double);
  if (c.imex_work_bytes < need) {
    if (c.d_imex_work) FCW_HIP(hipFree(c.d_imex_work));
    c.d_imex_work = nullptr;
    c.imex_work_bytes = 0;
    FCW_HIP(hipMalloc(&c.d_imex_work, need));
    c.imex_work_bytes = need;
  }
  double* bv = c.d_imex_work;
  double* uold = bv + nvp;
  double* dold = uold + nvp;
  double* upred = dold + nvp;
  double* part = upred + nvp;
  const unsigned gw = (unsigned)((nc + 15) / 16);  // 16 lanes per implicit row
  const unsigned gb = blocks_for(nv);
  ImexUpd e{};
  e.u = u;
  e.d = d;
  e.dofs = c.d_imex_dofs;
  e.uold = uold;
  e.dold = dold;
  e.v = v_c;
  e.a = a_c;
  e.upred = upred;
  e.ndof = ndof;
  e.dt = dt;
  auto kc_rhs = [&](const double* uimp, double t) {
    imex_kc_rhs_kernel<<<gw, 256, 0, c.stream>>>(
        c.d_imex_kptr, c.d_imex_kcol, c.d_imex_kval, u, uimp, c.d_imex_dofs, c.d_src, nc, ndof,
        c.nnodes, nrhs, c.dim, c.p, c.npts[0], c.npts[1], t, c.d_imex_cpos, bv);
  };
  fcw_status st;
  if (nc > 0) {
    // the implicit DOFs' state at the call's start; the fused updates keep it afterwards
    imex_gather_kernel<<<gb, 256, 0, c.stream>>>(u, c.d_imex_dofs, nc, ndof, nrhs, uold);
    if (consistent)
      imex_gather_kernel<<<gb, 256, 0, c.stream>>>(d, c.d_imex_dofs, nc, ndof, nrhs, dold);
  }
  if (consistent) {
    // central differences with the consistent cut-DOF mass: a = (M^cc)^{-1} (F - K^c u)
    // on the implicit DOFs (from u_k, before the explicit step overwrites it), the
    // lumped diagonal elsewhere
    for (int k = 0; k < nsteps; ++k) {
      const double t = t0 + k * dt;
      const int first = start && k == 0;
      if (nc > 0) {
        kc_rhs(uold, t);
        symp_tiles(c, c.d_imex_mp, bv, nrhs, part);
      }
      if ((st = run_steps(c, c.tile_choice, nrhs, u, d, c.d_ubuf, t, dt, 1, first))) return st;
      if (nc > 0) {
        e.w = (first ? 0.5 : 1.0) * dt * dt;
        symp_finish<kUpdCons>(c, part, nrhs, e);
      }
      FCW_HIP(hipGetLastError());
    }
    return FCW_OK;
  }
  if (start && nc > 0) {
    // a_0 = (M^cc)^{-1} (F_0 - K^c u_0) on the implicit DOFs
    kc_rhs(uold, t0);
    symp_tiles(c, c.d_imex_mp, bv, nrhs, part);
    symp_finish<kUpdStore>(c, part, nrhs, e);
  }
  // the first predictor; each corrector leaves the next one
  if (nc > 0) imex_predict_kernel<<<gb, 256, 0, c.stream>>>(uold, v_c, a_c, nv, dt, upred);
  for (int k = 0; k < nsteps; ++k) {
    const double t = t0 + k * dt;
    // explicit DOFs: one central-difference step of the explicit solver
    if ((st = run_steps(c, c.tile_choice, nrhs, u, d, c.d_ubuf, t, dt, 1, (start && k == 0))))
      return st;
    if (nc == 0) continue;
    // K^c u_p: the explicit DOFs' new values with the predictor on the implicit DOFs
    kc_rhs(upred, t + dt);
    symp_tiles(c, c.d_imex_sp, bv, nrhs, part);
    symp_finish<kUpdImex>(c, part, nrhs, e);
    FCW_HIP(hipGetLastError());
  }
  return FCW_OK;
}

}  // namespace fcw
