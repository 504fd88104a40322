// Setup kernels of the spectral cell method, all in FP64 on the device:
//  - 1-D GLL / GL rules (Sec. 2.2), uncut reference element and GLL lumped mass,
//  - cell classification against the voids (Sec. 2.2: cells outside the physical
//    domain are dropped) and compaction of the cut cells,
//  - space-tree quadrature of every cut cell (Sec. 2.2) giving K_e and M^o_e,
//  - eigenvalue stabilisation (Sec. 2.6) + HRZ lumping (Sec. 2.4) of the cut-cell
//    masses by a batched parallel-ordering Jacobi eigensolver,
//  - assembly of the diagonal mass and packing of the per-step operands.
// Geometric predicates and quadrature coordinates are evaluated with contraction
// disabled so that they follow plain IEEE double arithmetic step by step.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include <cstring>

#include "common.h"
#include "cube.h"

namespace fcw {

// --------------------------------------------------------------------------------
// 1-D rules
// --------------------------------------------------------------------------------

__device__ static void legendre_pair(int n, double x, double& pn, double& pn1) {
  // P_n(x) and P_{n-1}(x) by the three-term recurrence
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// Gauss-Legendre rule of n points on [-1, 1]: the roots of P_n by Newton's method.
__device__ static void gl_rule(int n, double* xs, double* ws) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = -cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pn1;
      legendre_pair(n, x, pn, pn1);
      double d1 = n * (pn1 - x * pn) / (1.0 - x * x);
      double dx = pn / d1;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double pn, pn1;
    legendre_pair(n, x, pn, pn1);
    double d1 = n * (pn1 - x * pn) / (1.0 - x * x);
    xs[i] = x;
    ws[i] = 2.0 / ((1.0 - x * x) * d1 * d1);
  }
}

__global__ void ref_tables_kernel(RefTables* tab, int p) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double pi = 3.14159265358979323846;
  // GLL: -1, +1 and the roots of P_p'; Newton on P_p' with P_p'' from the ODE.
  tab->gll_x[0] = -1.0;
  tab->gll_x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, pn1;
      legendre_pair(p, x, pn, pn1);
      double d1 = p * (pn1 - x * pn) / (1.0 - x * x);
      double d2 = (2.0 * x * d1 - p * (p + 1.0) * pn) / (1.0 - x * x);
      double dx = d1 / d2;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    tab->gll_x[i] = x;
  }
  for (int i = 0; i <= p; ++i) {
    double pn, pn1;
    legendre_pair(p, tab->gll_x[i], pn, pn1);
    tab->gll_w[i] = 2.0 / (p * (p + 1.0) * pn * pn);
  }
  // GL with n = p+1 points
  gl_rule(p + 1, tab->gl_x, tab->gl_w);
}

// Lagrange polynomials on the GLL nodes and their derivatives at x (product rule).
template <int NP1>
__device__ static void lagrange_1d(const double* nodes, double x, double* L, double* dL) {
#pragma clang fp contract(off)
  for (int i = 0; i < NP1; ++i) {
    double v = 1.0;
    for (int j = 0; j < NP1; ++j)
      if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    L[i] = v;
    double dv = 0.0;
    for (int k = 0; k < NP1; ++k) {
      if (k == i) continue;
      double t = 1.0 / (nodes[i] - nodes[k]);
      for (int j = 0; j < NP1; ++j)
        if (j != i && j != k) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
      dv += t;
    }
    dL[i] = dv;
  }
}

__global__ void gll_lumped_kernel(const RefTables* tab, int dim, int p, double h, double rho,
                                  double* lref) {
  int ns = 1;
  for (int k = 0; k < dim; ++k) ns *= (p + 1);
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ns) return;
  double m = rho;
  for (int k = 0; k < dim; ++k) m *= 0.5 * h;
  int r = a;
  for (int k = 0; k < dim; ++k) {
    m *= tab->gll_w[r % (p + 1)];
    r /= (p + 1);
  }
  lref[a] = m;
}

// --------------------------------------------------------------------------------
// Classification
// --------------------------------------------------------------------------------

struct Grid {
  int dim;
  int n[3];
  double lo[3];
  double h;
};

__device__ static void cell_box(const Grid& g, int64_t cell, double* blo, double* bhi) {
#pragma clang fp contract(off)
  int64_t r = cell;
  for (int k = 0; k < g.dim; ++k) {
    int64_t i = r % g.n[k];
    r /= g.n[k];
    blo[k] = g.lo[k] + (double)i * g.h;
    bhi[k] = g.lo[k] + (double)(i + 1) * g.h;
  }
}

// (meets, contained) of box [lo,hi] and ball (c, r): squared distance to the box
// below r^2, squared distance to the farthest corner at most r^2.
__device__ static void box_ball(int dim, const double* lo, const double* hi, const double* c,
                                double r, bool& meets, bool& contained) {
#pragma clang fp contract(off)
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    double gap = fmax(fmax(lo[k] - c[k], 0.0), c[k] - hi[k]);
    double far = fmax(fabs(c[k] - lo[k]), fabs(hi[k] - c[k]));
    dmin2 = dmin2 + gap * gap;
    dmax2 = dmax2 + far * far;
  }
  meets = dmin2 < r * r;
  contained = dmax2 <= r * r;
}

__global__ void classify_kernel(Grid g, CubeGeo cube, int64_t ncell, int nvoids,
                                const double* vc, const double* vr, int8_t* cls,
                                int32_t* iscut, int32_t* nmeet) {
  int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  double blo[3], bhi[3];
  cell_box(g, cell, blo, bhi);
  bool any = false, inside = false;
  if (cube.on) cube_box(cube, blo, bhi, any, inside);
  int cnt = 0;
  for (int v = 0; v < nvoids; ++v) {
    bool m, c;
    box_ball(g.dim, blo, bhi, vc + (int64_t)v * g.dim, vr[v], m, c);
    inside |= c;
    any |= m;
    cnt += m ? 1 : 0;
  }
  int8_t k = inside ? kClsOut : (any ? kClsCut : kClsUncut);
  cls[cell] = k;
  iscut[cell] = (k == kClsCut) ? 1 : 0;
  nmeet[cell] = (k == kClsCut) ? cnt : 0;
}

__global__ void compact_cut_kernel(Grid g, int64_t ncell, int nvoids, const double* vc,
                                   const double* vr, const int8_t* cls, const int32_t* cutpos,
                                   const int32_t* voff, int32_t* info, int32_t* cut_cells,
                                   int32_t* vptr, int32_t* vidx) {
  int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  int8_t k = cls[cell];
  if (k == kClsOut) { info[cell] = kInfoOut; return; }
  if (k == kClsUncut) { info[cell] = kInfoUncut; return; }
  int q = cutpos[cell];
  info[cell] = q;
  cut_cells[q] = (int32_t)cell;
  int off = voff[cell];
  vptr[q] = off;
  double blo[3], bhi[3];
  cell_box(g, cell, blo, bhi);
  for (int v = 0; v < nvoids; ++v) {
    bool m, c;
    box_ball(g.dim, blo, bhi, vc + (int64_t)v * g.dim, vr[v], m, c);
    if (m) vidx[off++] = v;
  }
}

// ---- deterministic exclusive scan of int32 (two levels, 4096 items per block) ----
constexpr int kScanThreads = 1024, kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ static int block_exclusive_scan_1024(int v, int* sh) {
  // Hillis-Steele inclusive scan over 1024 threads, returns the exclusive prefix.
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(1024) void scan_block_kernel(const int32_t* in, int32_t* out,
                                                          int32_t* sums, int64_t n) {
  __shared__ int sh[kScanThreads];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int tot = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    tot += v[i];
  }
  int pre = block_exclusive_scan_1024(tot, sh);
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = pre;
    pre += v[i];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = pre;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(int32_t* sums, int nblocks,
                                                         int32_t* total) {
  __shared__ int sh[kScanThreads];
  int carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += kScanThreads) {
    int i = b0 + threadIdx.x;
    int v = (i < nblocks) ? sums[i] : 0;
    int pre = block_exclusive_scan_1024(v, sh);
    if (i < nblocks) sums[i] = pre + carry;
    // total of this chunk: last thread's inclusive value
    if (threadIdx.x == kScanThreads - 1) sh[0] = pre + v;
    __syncthreads();
    carry += sh[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = carry;
}

__global__ void scan_add_kernel(int32_t* out, const int32_t* sums, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / kScanBlock];
}

// exclusive scan of n ints on the stream; writes the total to *total_host (syncs).
fcw_status exclusive_scan(Ctx& c, const int32_t* in, int32_t* out, int64_t n,
                          int32_t* total_host) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb < 1) nb = 1;
  int32_t* sums = nullptr;
  FCW_HIP(hipMallocAsync((void**)&sums, (nb + 1) * sizeof(int32_t), c.stream));
  scan_block_kernel<<<(unsigned)nb, kScanThreads, 0, c.stream>>>(in, out, sums, n);
  scan_sums_kernel<<<1, kScanThreads, 0, c.stream>>>(sums, (int)nb, sums + nb);
  scan_add_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c.stream>>>(out, sums, n);
  FCW_HIP(hipGetLastError());
  FCW_HIP(hipMemcpyAsync(total_host, sums + nb, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  FCW_HIP(hipFreeAsync(sums, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  return FCW_OK;
}

static Grid make_grid(const Ctx& c) {
  Grid g;
  g.dim = c.dim;
  g.h = c.h;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = c.ncells[k];
    g.lo[k] = c.lo[k];
  }
  return g;
}

fcw_status setup_reference(Ctx& c) {
  ref_tables_kernel<<<1, 64, 0, c.stream>>>(c.d_tab, c.p);
  gll_lumped_kernel<<<(c.n_s + 255) / 256, 256, 0, c.stream>>>(c.d_tab, c.dim, c.p, c.h,
                                                              c.rho, c.d_lref);
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

fcw_status setup_classify(Ctx& c) {
  Grid g = make_grid(c);
  const int64_t n = c.ncell_total;
  int32_t *iscut = nullptr, *nmeet = nullptr, *cutpos = nullptr, *voff = nullptr;
  FCW_HIP(hipMallocAsync((void**)&iscut, n * 4, c.stream));
  FCW_HIP(hipMallocAsync((void**)&nmeet, n * 4, c.stream));
  FCW_HIP(hipMallocAsync((void**)&cutpos, n * 4, c.stream));
  FCW_HIP(hipMallocAsync((void**)&voff, n * 4, c.stream));
  const unsigned nb = (unsigned)((n + 255) / 256);
  classify_kernel<<<nb, 256, 0, c.stream>>>(g, c.cube, n, c.nvoids, c.d_void_c, c.d_void_r, c.d_cls,
                                            iscut, nmeet);
  FCW_HIP(hipGetLastError());
  int32_t ncut = 0, nv = 0;
  fcw_status st = exclusive_scan(c, iscut, cutpos, n, &ncut);
  if (st != FCW_OK) return st;
  st = exclusive_scan(c, nmeet, voff, n, &nv);
  if (st != FCW_OK) return st;
  c.n_cut_cand = ncut;
  const int64_t nc = ncut > 0 ? ncut : 1;
  FCW_HIP(hipMalloc((void**)&c.d_cut_cells, nc * 4));
  FCW_HIP(hipMalloc((void**)&c.d_cut_vptr, (nc + 1) * 4));
  FCW_HIP(hipMalloc((void**)&c.d_cut_vidx, (nv > 0 ? nv : 1) * 4));
  FCW_HIP(hipMalloc((void**)&c.d_all_void, nc * 4));
  c.footprint += nc * 4 * 3 + (nv > 0 ? nv : 1) * 4;
  compact_cut_kernel<<<nb, 256, 0, c.stream>>>(g, n, c.nvoids, c.d_void_c, c.d_void_r,
                                               c.d_cls, cutpos, voff, c.d_info, c.d_cut_cells,
                                               c.d_cut_vptr, c.d_cut_vidx);
  FCW_HIP(hipGetLastError());
  FCW_HIP(hipMemcpyAsync(c.d_cut_vptr + ncut, &nv, 4, hipMemcpyHostToDevice, c.stream));
  FCW_HIP(hipFreeAsync(iscut, c.stream));
  FCW_HIP(hipFreeAsync(nmeet, c.stream));
  FCW_HIP(hipFreeAsync(cutpos, c.stream));
  FCW_HIP(hipFreeAsync(voff, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  return FCW_OK;
}

// --------------------------------------------------------------------------------
// Space-tree quadrature
// --------------------------------------------------------------------------------

// Box record of the tree: level (4 bits) | kind (2 bits) | ix, iy, iz (8 bits each).
enum { kKindAlpha = 0, kKindOne = 1, kKindLeaf = 2, kKindCut = 3 };
__device__ static inline uint32_t box_pack(int lvl, int kind, int ix, int iy, int iz) {
  return (uint32_t)lvl | ((uint32_t)kind << 4) | ((uint32_t)ix << 6) | ((uint32_t)iy << 14) |
         ((uint32_t)iz << 22);
}
__device__ static inline void box_unpack(uint32_t b, int& lvl, int& kind, int* ix) {
  lvl = b & 15;
  kind = (b >> 4) & 3;
  ix[0] = (b >> 6) & 255;
  ix[1] = (b >> 14) & 255;
  ix[2] = (b >> 22) & 255;
}

// bounds of a tree box by replaying the midpoint bisection from the cell box
__device__ static void tree_box_bounds(int dim, const double* clo, const double* chi, int lvl,
                                       const int* ix, double* lo, double* hi) {
#pragma clang fp contract(off)
  for (int k = 0; k < dim; ++k) {
    double a = clo[k], b = chi[k];
    for (int s = lvl - 1; s >= 0; --s) {
      double mid = 0.5 * (a + b);
      if ((ix[k] >> s) & 1) a = mid; else b = mid;
    }
    lo[k] = a;
    hi[k] = b;
  }
}

struct TreeArgs {
  Grid g;
  CubeGeo cube;
  const int32_t* cut_cells;
  const int32_t* vptr;
  const int32_t* vidx;
  const double* vc;
  const double* vr;
  const RefTables* tab;
  double alpha, rho, c2, lam, mu;
  int depth;
  int reference;  // 1: integrate the full cell [0,h]^d with no voids (one block)
  double* kout;
  double* mout;
  int32_t* all_void;
};

constexpr int kTreeThreads = 256;
constexpr int kTreeMaxBoxes = 1024;
constexpr int kTreeBatch = 64;

// block-wide exclusive scan of two counters (256 threads)
__device__ static void scan2_256(int a, int b, int& pa, int& pb, int& ta, int& tb, int* sh) {
  int t = threadIdx.x;
  sh[t] = a;
  sh[256 + t] = b;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int xa = (t >= off) ? sh[t - off] : 0;
    int xb = (t >= off) ? sh[256 + t - off] : 0;
    __syncthreads();
    sh[t] += xa;
    sh[256 + t] += xb;
    __syncthreads();
  }
  pa = sh[t] - a;
  pb = sh[256 + t] - b;
  ta = sh[255];
  tb = sh[511];
  __syncthreads();
}

// ---- leaf integration of 3-D scalar cut cells on the matrix cores ----
// Over a batch of leaf points the leaf parts are K += sum_(q,b) w1_q G_b(q) G_b(q)^T and
// M += sum_q w0_q N(q) N(q)^T: products of an (n_s x kappa) and a (kappa x n_s) operand
// with kappa the (point, direction) rows.  The n_s x n_s outputs (padded to NT x NT tiles
// of 16) keep their upper tiles in mfma_f64_16x16x4 accumulators, K tiles then M tiles,
// tile t on wave t mod 4.
typedef double tree_f64x4 __attribute__((ext_vector_type(4)));

template <int NT>
struct TreeTiles {
  static constexpr int NUT = NT * (NT + 1) / 2;
  int I[2 * NUT], J[2 * NUT], mat[2 * NUT];
  constexpr TreeTiles() : I(), J(), mat() {
    int t = 0;
    for (int m = 0; m < 2; ++m)
      for (int jj = 0; jj < NT; ++jj)
        for (int ii = 0; ii <= jj; ++ii) {
          I[t] = ii;
          J[t] = jj;
          mat[t] = m;
          ++t;
        }
  }
};

// one batch: gk rows (point, direction) and nk rows (point) of LS doubles, weights
// wq[point] = (w0, w1); lane l16 + 16 k4 holds operand row 4 ks + k4, column 16 blk + l16
template <int NT, int W, int NBQ, int LS, int TPW>
__device__ static __attribute__((always_inline)) void tree_leaf_mfma(const double* gk, const double* nk, const double* wq,
                                      int lane, tree_f64x4 (&acc)[TPW]) {
  constexpr TreeTiles<NT> tt{};
  constexpr int NTILE = 2 * TreeTiles<NT>::NUT;
  const int l16 = lane & 15, k4 = lane >> 4;
  // K: 3 NBQ rows
#pragma unroll 1
  for (int ks = 0; ks < 3 * NBQ / 4; ++ks) {
    const int r = 4 * ks + k4;
    const double w = wq[(r / 3) * 2 + 1];
    double bf[NT], af[NT];
#pragma unroll
    for (int jb = 0; jb < NT; ++jb) {
      bf[jb] = gk[r * LS + jb * 16 + l16];
      af[jb] = w * bf[jb];
    }
#pragma unroll
    for (int m = 0; m < TPW; ++m) {
      const int t = W + 4 * m;
      if (t < NTILE && tt.mat[t] == 0)
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[tt.I[t]], bf[tt.J[t]], acc[m], 0, 0, 0);
    }
  }
  // M: NBQ rows
#pragma unroll 1
  for (int ks = 0; ks < NBQ / 4; ++ks) {
    const int r = 4 * ks + k4;
    const double w = wq[r * 2];
    double bf[NT], af[NT];
#pragma unroll
    for (int jb = 0; jb < NT; ++jb) {
      bf[jb] = nk[r * LS + jb * 16 + l16];
      af[jb] = w * bf[jb];
    }
#pragma unroll
    for (int m = 0; m < TPW; ++m) {
      const int t = W + 4 * m;
      if (t < NTILE && tt.mat[t] == 1)
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[tt.I[t]], bf[tt.J[t]], acc[m], 0, 0, 0);
    }
  }
}

// adds the wave's tiles (times c^2 rho for K, rho for M) to the full symmetric K and M
template <int NT, int W, int NS, int TPW>
__device__ static __attribute__((always_inline)) void tree_leaf_store(double* K, double* M, double krho, double rho, int lane,
                                       const tree_f64x4 (&acc)[TPW]) {
  constexpr TreeTiles<NT> tt{};
  constexpr int NTILE = 2 * TreeTiles<NT>::NUT;
  const int l16 = lane & 15, k4 = lane >> 4;
#pragma unroll
  for (int m = 0; m < TPW; ++m) {
    const int t = W + 4 * m;
    if (t >= NTILE) continue;
    double* D = tt.mat[t] == 0 ? K : M;
    const double sc = tt.mat[t] == 0 ? krho : rho;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tt.I[t] * 16 + 4 * r + k4, j = tt.J[t] * 16 + l16;
      if (i < NS && j < NS) {
        const double v = sc * acc[m][r];
        D[i * NS + j] += v;
        if (tt.I[t] != tt.J[t]) D[j * NS + i] += v;
      }
    }
  }
}

template <int DIM, int P, int NCOMP>
__global__ __launch_bounds__(kTreeThreads) void tree_integrate_kernel(TreeArgs a) {
#pragma clang fp contract(off)
  constexpr int NP1 = P + 1;
  constexpr int NS = ipow(NP1, DIM);
  constexpr int NPB = NS;  // GL points per box
  constexpr int NENT = NS * (NS + 1) / 2;
  constexpr int EPT = (NENT + kTreeThreads - 1) / kTreeThreads;
  constexpr int NG = (NCOMP == 1) ? 1 : DIM * DIM;
  constexpr int PD = 2 + 2 * DIM * NP1;  // per point: w_mass, w_stiff, L[DIM][NP1], dL[DIM][NP1]
  // leaf points are taken NBQ at a time; each point's shape values N[NS] and reference
  // gradients G[DIM][NS] are formed once (PDQ doubles with the two weights), so the
  // per-entry loop reads two values per function instead of re-forming the products
  constexpr int PDQ = 2 + (1 + DIM) * NS;
  // 3-D scalar cells integrate their leaves on the matrix cores (tree_leaf_mfma)
  constexpr bool MFL = DIM == 3 && NCOMP == 1;
  constexpr int NT = (NS + 15) / 16;
  constexpr int LS = (NT % 2 == 0) ? NT * 16 + 16 : NT * 16;  // row stride: 2-way banks
  constexpr int TPW = (2 * TreeTiles<NT>::NUT + 3) / 4;
  constexpr int NBQ_ = MFL ? (NT >= 8 ? 8 : 16) : (32 * 1024) / (PDQ * 8);
  constexpr int NBQ = NBQ_ < 1 ? 1 : (NBQ_ > kTreeBatch ? kTreeBatch : NBQ_);
  static_assert(!MFL || NBQ % 4 == 0, "whole k-steps of four operand rows");

  __shared__ uint32_t lst[2][kTreeMaxBoxes];
  __shared__ uint32_t outl[kTreeMaxBoxes];
  __shared__ int scan_sh[512];
  __shared__ double pts[NBQ * PD];
  __shared__ double ptq[MFL ? NBQ * (4 * LS + 2) : NBQ * PDQ];
  __shared__ int s_ncur, s_nout;

  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  double clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
  int vbeg = 0, vend = 0;
  if (a.reference) {
    for (int k = 0; k < DIM; ++k) { clo[k] = 0.0; chi[k] = a.g.h; }
  } else {
    cell_box(a.g, a.cut_cells[q], clo, chi);
    vbeg = a.vptr[q];
    vend = a.vptr[q + 1];
  }
  const double* gll = a.tab->gll_x;

  // ---- breadth-first construction of the tree, deterministic order ----
  if (tid == 0) {
    lst[0][0] = box_pack(0, kKindCut, 0, 0, 0);
    s_ncur = 1;
    s_nout = 0;
  }
  __syncthreads();
  int cur = 0;
  for (int lvl = 0; lvl <= a.depth; ++lvl) {
    const int ncur = s_ncur;
    int nnext = 0;
    for (int base = 0; base < ncur; base += kTreeThreads) {
      int i = base + tid;
      int kind = -1;
      int ix[3] = {0, 0, 0};
      if (i < ncur) {
        int l, kd;
        box_unpack(lst[cur][i], l, kd, ix);
        double lo[3], hi[3];
        tree_box_bounds(DIM, clo, chi, lvl, ix, lo, hi);
        bool any = false, inside = false;
        if (a.cube.on && !a.reference) cube_box(a.cube, lo, hi, any, inside);
        for (int v = vbeg; v < vend; ++v) {
          int vi = a.vidx[v];
          bool m, cc;
          box_ball(DIM, lo, hi, a.vc + (int64_t)vi * DIM, a.vr[vi], m, cc);
          inside |= cc;
          any |= m;
        }
        kind = inside ? kKindAlpha : (any ? (lvl < a.depth ? kKindCut : kKindLeaf) : kKindOne);
      }
      int nout_i = (kind >= 0 && kind != kKindCut) ? 1 : 0;
      int nch_i = (kind == kKindCut) ? (1 << DIM) : 0;
      int po, pc, to, tc;
      scan2_256(nout_i, nch_i, po, pc, to, tc, scan_sh);
      const int nout0 = s_nout;
      if (nout_i) outl[nout0 + po] = box_pack(lvl, kind, ix[0], ix[1], ix[2]);
      if (nch_i) {
        for (int ch = 0; ch < (1 << DIM); ++ch) {
          int cx = 2 * ix[0] + (ch & 1);
          int cy = 2 * ix[1] + ((ch >> 1) & 1);
          int cz = 2 * ix[2] + ((ch >> 2) & 1);
          // child order: x bit slowest, matching lexicographic (x, y, z) corner order
          int corder = 0;
          for (int k = 0; k < DIM; ++k) corder = corder * 2 + ((ch >> k) & 1);
          int pos = nnext + pc + corder;
          if (pos < kTreeMaxBoxes) lst[cur ^ 1][pos] = box_pack(lvl + 1, kKindCut, cx, cy, cz);
        }
      }
      __syncthreads();
      if (tid == 0) s_nout = nout0 + to;
      nnext += tc;
      __syncthreads();
    }
    if (tid == 0) s_ncur = nnext;
    cur ^= 1;
    __syncthreads();
  }
  const int nout = s_nout;

  // ---- integration ----
  int eij[EPT];  // row | column << 16 of each entry of this thread
  double accM[EPT], accG[EPT][NG];
  for (int e = 0; e < EPT; ++e) {
    int lin = tid + e * kTreeThreads;
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= lin) ++j;
    int i = lin - j * (j + 1) / 2;
    eij[e] = (lin < NENT) ? (i | (j << 16)) : 0;
    accM[e] = 0.0;
    for (int g = 0; g < NG; ++g) accG[e][g] = 0.0;
  }
  const double jac = 2.0 / a.g.h;

  // ---- boxes of constant alpha (all material or all void): the integrands separate,
  // so each box adds products of 1-D integrals over its intervals (GL (p+1) per
  // direction: exact, as the pointwise rule is on such a box) ----
  __shared__ double t1[DIM][3][NP1 * NP1];  // per direction: m1, d1, g1 of the box
  __shared__ int s_nleaf;
  for (int b = 0; b < nout; ++b) {
    int lvl, kind, ix[3];
    box_unpack(outl[b], lvl, kind, ix);
    if (kind == kKindLeaf) continue;
    double lo[3], hi[3];
    tree_box_bounds(DIM, clo, chi, lvl, ix, lo, hi);
    if (tid < DIM * NP1 * NP1) {
      const int k = tid / (NP1 * NP1), i = (tid / NP1) % NP1, jj = tid % NP1;
      const double half = 0.5 * (hi[k] - lo[k]);
      double m = 0.0, dd = 0.0, g = 0.0;
      for (int qp = 0; qp < NP1; ++qp) {
        const double x = lo[k] + (a.tab->gl_x[qp] + 1.0) * half;
        const double xi = 2.0 * (x - clo[k]) / a.g.h - 1.0;
        double L[NP1], dL[NP1];
        lagrange_1d<NP1>(gll, xi, L, dL);
        const double w = a.tab->gl_w[qp] * half;
        m += w * L[i] * L[jj];
        dd += w * (jac * dL[i]) * (jac * dL[jj]);
        g += w * (jac * dL[i]) * L[jj];
      }
      t1[k][0][i * NP1 + jj] = m;
      t1[k][1][i * NP1 + jj] = dd;
      t1[k][2][i * NP1 + jj] = g;
    }
    __syncthreads();
    const double al = (kind == kKindAlpha) ? a.alpha : 1.0;
    for (int e = 0; e < EPT; ++e) {
      if (tid + e * kTreeThreads >= NENT) break;
      int ia[3] = {0, 0, 0}, ja[3] = {0, 0, 0};
      int ri = eij[e] & 0xFFFF, rj = eij[e] >> 16;
      for (int k = 0; k < DIM; ++k) {
        ia[k] = ri % NP1; ri /= NP1;
        ja[k] = rj % NP1; rj /= NP1;
      }
      double mm = al;
      for (int k = 0; k < DIM; ++k) mm *= t1[k][0][ia[k] * NP1 + ja[k]];
      accM[e] += mm;
      for (int bb = 0; bb < DIM; ++bb)
        for (int c2 = 0; c2 < DIM; ++c2) {
          if (NCOMP == 1 && bb != c2) continue;
          // d/dx_bb of N_i times d/dx_c2 of N_j, direction by direction
          double v = al;
          for (int k = 0; k < DIM; ++k) {
            if (k == bb && k == c2) v *= t1[k][1][ia[k] * NP1 + ja[k]];
            else if (k == bb) v *= t1[k][2][ia[k] * NP1 + ja[k]];
            else if (k == c2) v *= t1[k][2][ja[k] * NP1 + ia[k]];
            else v *= t1[k][0][ia[k] * NP1 + ja[k]];
          }
          accG[e][NCOMP == 1 ? 0 : bb * DIM + c2] += v;
        }
    }
    __syncthreads();
  }
  // the leaves (cut at the finest level) keep the pointwise rule with alpha per point
  if (tid == 0) {
    int nl = 0;
    for (int b = 0; b < nout; ++b) {
      int lvl, kind, ix[3];
      box_unpack(outl[b], lvl, kind, ix);
      if (kind == kKindLeaf) lst[0][nl++] = outl[b];
    }
    s_nleaf = nl;
  }
  __syncthreads();
  const uint32_t* leafl = lst[0];
  const int npts_total = s_nleaf * NPB;
  // weights, 1-D Lagrange values and derivatives of the leaf points pb .. pb + NBQ - 1
  auto prep_points = [&](int pb) {
    if (tid < NBQ) {
      int ip = pb + tid;
      double* d = pts + tid * PD;
      if (ip < npts_total) {
        int bi = ip / NPB, qi = ip % NPB;
        int lvl, kind, ix[3];
        box_unpack(leafl[bi], lvl, kind, ix);
        double lo[3], hi[3];
        tree_box_bounds(DIM, clo, chi, lvl, ix, lo, hi);
        double x[3], w = 1.0;
        int r = qi;
        for (int k = 0; k < DIM; ++k) {
          int m = r % NP1;
          r /= NP1;
          double half = 0.5 * (hi[k] - lo[k]);
          x[k] = lo[k] + (a.tab->gl_x[m] + 1.0) * half;
          w = w * (a.tab->gl_w[m] * half);
        }
        double al = 1.0;
        if (kind == kKindAlpha) {
          al = a.alpha;
        } else if (kind == kKindLeaf) {
          if (a.cube.on && cube_point_outside(a.cube, x)) al = a.alpha;
          for (int v = vbeg; v < vend && al == 1.0; ++v) {
            int vi = a.vidx[v];
            const double* cc = a.vc + (int64_t)vi * DIM;
            double d2 = 0.0;
            for (int k = 0; k < DIM; ++k) d2 = d2 + (x[k] - cc[k]) * (x[k] - cc[k]);
            if (d2 < a.vr[vi] * a.vr[vi]) { al = a.alpha; break; }
          }
        }
        d[0] = w * al;
        d[1] = w * al * jac * jac;
        for (int k = 0; k < DIM; ++k) {
          double xi = 2.0 * (x[k] - clo[k]) / a.g.h - 1.0;
          lagrange_1d<NP1>(gll, xi, d + 2 + k * NP1, d + 2 + DIM * NP1 + k * NP1);
        }
      } else {
        for (int k = 0; k < PD; ++k) d[k] = 0.0;
      }
    }
  };
  auto write_out = [&]() {
    constexpr int NL = NCOMP * NS;
    double* K = a.kout + (int64_t)q * NL * NL;
    double* M = a.mout + (int64_t)q * NS * NS;
    for (int e = 0; e < EPT; ++e) {
      if (tid + e * kTreeThreads >= NENT) break;
      const int i = eij[e] & 0xFFFF, j = eij[e] >> 16;
      const double m = a.rho * accM[e];
      M[i * NS + j] = m;
      M[j * NS + i] = m;
      if (NCOMP == 1) {
        const double k = a.c2 * a.rho * accG[e][0];
        K[i * NL + j] = k;
        K[j * NL + i] = k;
      } else {
        double tr = 0.0;
        for (int b = 0; b < DIM; ++b) tr += accG[e][b * DIM + b];
        for (int cc = 0; cc < NCOMP; ++cc)
          for (int ee = 0; ee < NCOMP; ++ee) {
            // K[(c,i),(e,j)] = lam G_ce[i][j] + mu G_ec[i][j] + mu delta_ce sum_a G_aa[i][j]
            double v = a.lam * accG[e][cc * DIM + ee] + a.mu * accG[e][ee * DIM + cc] +
                       (cc == ee ? a.mu * tr : 0.0);
            K[(cc * NS + i) * NL + ee * NS + j] = v;
            K[(ee * NS + j) * NL + cc * NS + i] = v;
          }
      }
    }
  };
  if constexpr (MFL) {
    // the constant boxes' sums go out first; the leaves are added on the matrix cores
    write_out();
    __syncthreads();
    double* gk = ptq;                    // [NBQ][DIM][LS]
    double* nk = ptq + NBQ * DIM * LS;   // [NBQ][LS]
    double* wq = ptq + NBQ * 4 * LS;     // [NBQ][2]
    const int wave = tid >> 6, lane = tid & 63;
    tree_f64x4 acc[TPW];
#pragma unroll
    for (int m = 0; m < TPW; ++m) acc[m] = tree_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int pb = 0; pb < npts_total; pb += NBQ) {
      prep_points(pb);
      __syncthreads();
      // operand rows: N and the reference gradients of every point (zero beyond n_s)
      for (int t = tid; t < NBQ * NT * 16; t += kTreeThreads) {
        const int qp = t / (NT * 16), an = t % (NT * 16);
        const double* d = pts + qp * PD;
        const double* L = d + 2;
        const double* dL = d + 2 + DIM * NP1;
        double Nv = 0.0, Gv[DIM];
        for (int b = 0; b < DIM; ++b) Gv[b] = 0.0;
        if (an < NS) {
          int ia[3] = {0, 0, 0};
          int ri = an;
          for (int k = 0; k < DIM; ++k) { ia[k] = ri % NP1; ri /= NP1; }
          Nv = 1.0;
          for (int k = 0; k < DIM; ++k) Nv *= L[k * NP1 + ia[k]];
          for (int b = 0; b < DIM; ++b) {
            double v = dL[b * NP1 + ia[b]];
            for (int k = 0; k < DIM; ++k) {
              if (k == b) continue;
              v *= L[k * NP1 + ia[k]];
            }
            Gv[b] = v;
          }
        }
        nk[qp * LS + an] = Nv;
        for (int b = 0; b < DIM; ++b) gk[(qp * DIM + b) * LS + an] = Gv[b];
        if (an == 0) {
          wq[qp * 2] = d[0];
          wq[qp * 2 + 1] = d[1];
        }
      }
      __syncthreads();
      switch (wave) {
        case 0: tree_leaf_mfma<NT, 0, NBQ, LS, TPW>(gk, nk, wq, lane, acc); break;
        case 1: tree_leaf_mfma<NT, 1, NBQ, LS, TPW>(gk, nk, wq, lane, acc); break;
        case 2: tree_leaf_mfma<NT, 2, NBQ, LS, TPW>(gk, nk, wq, lane, acc); break;
        default: tree_leaf_mfma<NT, 3, NBQ, LS, TPW>(gk, nk, wq, lane, acc); break;
      }
      __syncthreads();
    }
    double* Kq = a.kout + (int64_t)q * NS * NS;
    double* Mq = a.mout + (int64_t)q * NS * NS;
    const double krho = a.c2 * a.rho;
    switch (wave) {
      case 0: tree_leaf_store<NT, 0, NS, TPW>(Kq, Mq, krho, a.rho, lane, acc); break;
      case 1: tree_leaf_store<NT, 1, NS, TPW>(Kq, Mq, krho, a.rho, lane, acc); break;
      case 2: tree_leaf_store<NT, 2, NS, TPW>(Kq, Mq, krho, a.rho, lane, acc); break;
      default: tree_leaf_store<NT, 3, NS, TPW>(Kq, Mq, krho, a.rho, lane, acc); break;
    }
  } else {
    for (int pb = 0; pb < npts_total; pb += NBQ) {
      prep_points(pb);
      __syncthreads();
      // N_a = prod_k L_k(i_k(a)) and G_b,a = dL_b(i_b(a)) prod_{k != b} L_k(i_k(a)), products
      // taken in increasing k
      for (int t = tid; t < NBQ * NS; t += kTreeThreads) {
        const int qp = t / NS, an = t % NS;
        const double* d = pts + qp * PD;
        const double* L = d + 2;
        const double* dL = d + 2 + DIM * NP1;
        double* o = ptq + qp * PDQ;
        int ia[3] = {0, 0, 0};
        int ri = an;
        for (int k = 0; k < DIM; ++k) { ia[k] = ri % NP1; ri /= NP1; }
        double Nv = 1.0;
        for (int k = 0; k < DIM; ++k) Nv *= L[k * NP1 + ia[k]];
        o[2 + an] = Nv;
        for (int b = 0; b < DIM; ++b) {
          double v = dL[b * NP1 + ia[b]];
          for (int k = 0; k < DIM; ++k) {
            if (k == b) continue;
            v *= L[k * NP1 + ia[k]];
          }
          o[2 + (1 + b) * NS + an] = v;
        }
        if (an == 0) {
          o[0] = d[0];
          o[1] = d[1];
        }
      }
      __syncthreads();
      const int nb = min(NBQ, npts_total - pb);
      for (int e = 0; e < EPT; ++e) {
        if (tid + e * kTreeThreads >= NENT) break;
        const int ri = eij[e] & 0xFFFF, rj = eij[e] >> 16;
        double sm = 0.0;
        double sg[NG];
        for (int g = 0; g < NG; ++g) sg[g] = 0.0;
  #pragma unroll 1
        for (int qp = 0; qp < nb; ++qp) {
          // the entry's offsets are re-formed here (opaque to loop-invariant hoisting, which
          // would keep them live for every entry of the thread across the point loop)
          int oi = ri, oj = rj;
          asm volatile("" : "+v"(oi), "+v"(oj));
          const double* o = ptq + qp * PDQ;
          const double Ni = o[2 + oi], Nj = o[2 + oj];
          double gi[DIM], gj[DIM];
          for (int b = 0; b < DIM; ++b) {
            gi[b] = o[2 + (1 + b) * NS + oi];
            gj[b] = o[2 + (1 + b) * NS + oj];
          }
          sm += o[0] * Ni * Nj;
          if (NCOMP == 1) {
            double s = 0.0;
            for (int b = 0; b < DIM; ++b) s += gi[b] * gj[b];
            sg[0] += o[1] * s;
          } else {
            for (int b = 0; b < DIM; ++b)
              for (int c2 = 0; c2 < DIM; ++c2) sg[b * DIM + c2] += o[1] * gi[b] * gj[c2];
          }
        }
        accM[e] += sm;
        for (int g = 0; g < NG; ++g) accG[e][g] += sg[g];
      }
      __syncthreads();
    }

    write_out();
  }
  if (tid == 0 && !a.reference) {
    int allv = 1;
    for (int b = 0; b < nout; ++b) {
      int lvl, kind, ix[3];
      box_unpack(outl[b], lvl, kind, ix);
      if (kind != kKindAlpha) { allv = 0; break; }
    }
    a.all_void[q] = allv;
  }
}

template <int DIM, int P, int NCOMP>
static fcw_status launch_tree(Ctx& c, TreeArgs& ta, int nblocks) {
  tree_integrate_kernel<DIM, P, NCOMP><<<nblocks, kTreeThreads, 0, c.stream>>>(ta);
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

static fcw_status dispatch_tree(Ctx& c, TreeArgs& ta, int nblocks) {
#define FCW_TREE_CASE(D, PP, NC) \
  if (c.dim == D && c.p == PP && c.ncomp == NC) return launch_tree<D, PP, NC>(c, ta, nblocks);
  FCW_TREE_CASE(2, 1, 1) FCW_TREE_CASE(2, 2, 1) FCW_TREE_CASE(2, 3, 1) FCW_TREE_CASE(2, 4, 1)
  FCW_TREE_CASE(2, 5, 1) FCW_TREE_CASE(2, 6, 1)
  FCW_TREE_CASE(3, 1, 1) FCW_TREE_CASE(3, 2, 1) FCW_TREE_CASE(3, 3, 1) FCW_TREE_CASE(3, 4, 1)
  FCW_TREE_CASE(3, 1, 3) FCW_TREE_CASE(3, 2, 3) FCW_TREE_CASE(3, 3, 3)
#undef FCW_TREE_CASE
  set_error("tree integration not built for dim=%d p=%d ncomp=%d", c.dim, c.p, c.ncomp);
  return FCW_E_UNSUPPORTED;
}

fcw_status setup_integrate(Ctx& c) {
  TreeArgs ta{};
  ta.g = make_grid(c);
  ta.cube = c.cube;
  ta.cut_cells = c.d_cut_cells;
  ta.vptr = c.d_cut_vptr;
  ta.vidx = c.d_cut_vidx;
  ta.vc = c.d_void_c;
  ta.vr = c.d_void_r;
  ta.tab = c.d_tab;
  ta.alpha = c.alpha;
  ta.rho = c.rho;
  ta.c2 = c.c * c.c;
  ta.lam = c.E * c.nu / ((1.0 + c.nu) * (1.0 - 2.0 * c.nu));
  ta.mu = c.E / (2.0 * (1.0 + c.nu));
  ta.depth = c.depth;
  // reference (uncut) cell: one box integrated with constant 1
  ta.reference = 1;
  ta.kout = c.d_kref;
  ta.mout = c.d_mfull;
  ta.all_void = c.d_all_void;
  fcw_status st = dispatch_tree(c, ta, 1);
  if (st != FCW_OK) return st;
  if (c.n_cut_cand > 0) {
    ta.reference = 0;
    ta.kout = c.d_kcut;
    ta.mout = c.d_mcut;
    st = dispatch_tree(c, ta, (int)c.n_cut_cand);
    if (st != FCW_OK) return st;
  }
  return FCW_OK;
}

// --------------------------------------------------------------------------------
// Eigenvalue stabilisation + HRZ lumping (one workgroup per cut cell)
// --------------------------------------------------------------------------------

struct EvsArgs {
  int n, m;  // matrix order and its even padding
  const double* mcut;
  const double* mfull;
  double eps, f_lambda;
  int max_sweeps;
  double tol, tol_abs;  // pair (i, j) is resolved once |a_ij| <= max(tol sqrt|a_ii a_jj|, tol_abs max|a_kk|)
  double* lumped;
  double* margin;
  int32_t* fail;
};

constexpr int kEvsThreads = 256;

__device__ static double block_max_256(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) sh[t] = fmax(sh[t], sh[t + off]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ static double block_sum_256(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kEvsThreads) void evs_lump_kernel(EvsArgs a) {
  extern __shared__ double sm[];
  const int n = a.n, m = a.m, ld = m + 1;
  double* red = sm;                   // 256
  double* dg = red + kEvsThreads;     // n: original diagonal
  double* cs = dg + n;                // m/2 (c, s) pairs
  int* pq = (int*)(cs + m);           // m/2 (p, q) pairs
  double* A = (double*)(pq + m + (m & 1)) ;
  double* V = A + m * ld;             // A, V only when eps != 0
  const int tid = threadIdx.x;
  const int q = blockIdx.x;
  const double* Mo = a.mcut + (int64_t)q * n * n;

  double s_all = 0.0, s_diag = 0.0, mf = -1e300;
  for (int idx = tid; idx < n * n; idx += kEvsThreads) {
    double v = Mo[idx];
    s_all += v;
    if (idx / n == idx % n) s_diag += v;
    mf = fmax(mf, a.mfull[idx]);
  }
  for (int i = tid; i < n; i += kEvsThreads) dg[i] = Mo[i * n + i];
  if (a.eps != 0.0) {
    for (int idx = tid; idx < m * m; idx += kEvsThreads) {
      int i = idx / m, j = idx % m;
      A[i * ld + j] = (i < n && j < n) ? Mo[i * n + j] : 0.0;
      V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
  }
  const double me = block_sum_256(s_all, red);
  const double tr = block_sum_256(s_diag, red);
  const double maxmf = block_max_256(mf, red);
  __syncthreads();

  bool converged = true;
  double marg = 1e300;
  if (a.eps != 0.0) {
    converged = false;
    // cyclic Jacobi with a threshold: a relative test alone cannot be met by pairs of
    // eigenvalues far below the largest (their off-diagonal rounding comes from the
    // large entries), and such pairs do not move the split at f_lambda lambda_max
    for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
      double amax = 0.0;
      for (int i = tid; i < n; i += kEvsThreads) amax = fmax(amax, fabs(A[i * ld + i]));
      const double thr_abs = a.tol_abs * block_max_256(amax, red);
      double open = 0.0;
      for (int idx = tid; idx < n * n; idx += kEvsThreads) {
        int i = idx / n, j = idx % n;
        if (i < j) {
          double r = fabs(A[i * ld + j]);
          double thr = fmax(a.tol * sqrt(fabs(A[i * ld + i] * A[j * ld + j])), thr_abs);
          if (r > thr) open = 1.0;
        }
      }
      if (block_max_256(open, red) == 0.0) { converged = true; break; }
      for (int r = 0; r < m - 1; ++r) {
        if (tid < m / 2) {
          int p0, q0;
          if (tid == 0) { p0 = m - 1; q0 = r; }
          else { p0 = (r + tid) % (m - 1); q0 = (r - tid + (m - 1)) % (m - 1); }
          int pp = min(p0, q0), qq = max(p0, q0);
          double apq = A[pp * ld + qq];
          double c = 1.0, s = 0.0;
          const double app = A[pp * ld + pp], aqq = A[qq * ld + qq];
          if (fabs(apq) > fmax(a.tol * sqrt(fabs(app * aqq)), thr_abs)) {
            double tau = (aqq - app) / (2.0 * apq);
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
          pq[2 * tid] = pp;
          pq[2 * tid + 1] = qq;
          cs[2 * tid] = c;
          cs[2 * tid + 1] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < (m / 2) * m; idx += kEvsThreads) {
          int k = idx / m, col = idx % m;
          int pp = pq[2 * k], qq = pq[2 * k + 1];
          double c = cs[2 * k], s = cs[2 * k + 1];
          double ap = A[pp * ld + col], aq = A[qq * ld + col];
          A[pp * ld + col] = c * ap - s * aq;
          A[qq * ld + col] = s * ap + c * aq;
        }
        __syncthreads();
        for (int idx = tid; idx < (m / 2) * m; idx += kEvsThreads) {
          int k = idx / m, row = idx % m;
          int pp = pq[2 * k], qq = pq[2 * k + 1];
          double c = cs[2 * k], s = cs[2 * k + 1];
          double ap = A[row * ld + pp], aq = A[row * ld + qq];
          A[row * ld + pp] = c * ap - s * aq;
          A[row * ld + qq] = s * ap + c * aq;
          double vp = V[row * ld + pp], vq = V[row * ld + qq];
          V[row * ld + pp] = c * vp - s * vq;
          V[row * ld + qq] = s * vp + c * vq;
        }
        __syncthreads();
      }
    }
    // eigenvalues on the diagonal; small set S = {i : lambda_i < f_lambda lambda_max}
    double lmax = -1e300;
    for (int i = tid; i < n; i += kEvsThreads) lmax = fmax(lmax, A[i * ld + i]);
    lmax = block_max_256(lmax, red);
    double mg = 1e300;
    for (int i = tid; i < n; i += kEvsThreads) mg = fmin(mg, fabs(A[i * ld + i] / lmax - a.f_lambda));
    marg = -block_max_256(-mg, red);
    // diag(M~^s)_k = sum_{i in S} V_ki^2 ; red[k] holds it for k < n (n <= 256)
    double dk = 0.0;
    if (tid < n) {
      for (int i = 0; i < n; ++i)
        if (A[i * ld + i] < a.f_lambda * lmax) dk += V[tid * ld + i] * V[tid * ld + i];
    }
    __syncthreads();
    const double maxd = block_max_256(tid < n ? dk : 0.0, red);
    if (tid < n) {
      double ms = (maxd > 0.0) ? (maxmf / maxd) * dk : 0.0;
      a.lumped[(int64_t)q * n + tid] = me / tr * dg[tid] + a.eps * ms;
    }
  } else {
    for (int i = tid; i < n; i += kEvsThreads) a.lumped[(int64_t)q * n + i] = me / tr * dg[i];
  }
  if (tid == 0) {
    a.margin[q] = marg;
    a.fail[q] = converged ? 0 : 1;
  }
}

// Large cut cells (n_s too big for A and V of the Jacobi kernel in LDS, e.g. 3-D p=4):
// the same stabilised lumped diagonal through a tridiagonal reduction.  One workgroup
// per cut cell (grid-stride over the cells, one scratch slot per workgroup):
//  1. Householder reduction M^o = Q T Q^T with M^o in LDS; the reflectors go to the
//     workgroup's scratch slot in global memory;
//  2. implicit QL with shifts on T; waves 0 and 1 run the (scalar) recurrence each on
//     their own copy of T and rotate their own rows of the eigenvector matrix Z in LDS,
//     so no barrier is needed inside the iteration;
//  3. the columns of Z whose eigenvalues lie below f_lambda lambda_max are carried back
//     through the reflectors, X_S = Q Z_S, and diag(M~^s)_k = sum_{i in S} X_ki^2.
// Eigenvalues and the split come with the absolute accuracy of a symmetric eigensolver,
// as in the Jacobi kernel.
struct EvsBigArgs {
  int n, lda;
  const double* mcut;
  const double* mfull;
  double eps, f_lambda;
  int64_t ncand;
  double* scratch;  // [gridDim.x][n * n]
  double* lumped;
  double* margin;
  int32_t* fail;
};

__device__ static inline double hypot_scaled(double a, double b) {
  a = fabs(a);
  b = fabs(b);
  const double m = fmax(a, b), s = fmin(a, b);
  if (m == 0.0) return 0.0;
  const double r = s / m;
  return m * sqrt(1.0 + r * r);
}

__global__ __launch_bounds__(kEvsThreads) void evs_big_kernel(EvsBigArgs a) {
  extern __shared__ double smb[];
  const int n = a.n, lda = a.lda;
  double* A = smb;                    // n x lda: M^o, then Z
  double* red = A + n * lda;          // 256
  double* vb = red + kEvsThreads;     // n: reflector
  double* pb = vb + n;                // n: A v, then w
  double* dg = pb + n;                // n: original diagonal
  double* dq = dg + n;                // 2 x n: diagonal of T, one copy per wave
  double* eq = dq + 2 * n;            // 2 x n: off-diagonal of T
  double* dk = eq + 2 * n;            // n
  int* cols = (int*)(dk + n);         // n: columns of the small set
  __shared__ int nsmall, bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* hv = a.scratch + (int64_t)blockIdx.x * n * n;  // reflector k at k*n, tau at (n-1)*n+k

  for (int64_t q = blockIdx.x; q < a.ncand; q += gridDim.x) {
    const double* Mo = a.mcut + q * n * n;
    double s_all = 0.0, s_diag = 0.0, mf = -1e300;
    for (int idx = tid; idx < n * n; idx += kEvsThreads) {
      const int i = idx / n, j = idx % n;
      const double v = Mo[idx];
      s_all += v;
      if (i == j) s_diag += v;
      mf = fmax(mf, a.mfull[idx]);
      A[i * lda + j] = v;
    }
    for (int i = tid; i < n; i += kEvsThreads) dg[i] = Mo[i * n + i];
    const double me = block_sum_256(s_all, red);
    const double tr = block_sum_256(s_diag, red);
    const double maxmf = block_max_256(mf, red);

    // ---- 1. Householder reduction (A stays full and symmetric) ----
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1;  // length of the reflector
      double sq = 0.0;
      for (int i = tid; i < m; i += kEvsThreads) {
        const double x = A[(k + 1 + i) * lda + k];
        sq += x * x;
      }
      sq = block_sum_256(sq, red);
      const double x0 = A[(k + 1) * lda + k];
      const double nx = sqrt(sq);
      const double alpha = (x0 > 0.0) ? -nx : nx;
      const double vtv = sq - 2.0 * alpha * x0 + alpha * alpha;
      const double tau = (nx > 0.0 && vtv > 0.0) ? 2.0 / vtv : 0.0;
      for (int i = tid; i < m; i += kEvsThreads) {
        const double v = A[(k + 1 + i) * lda + k] - (i == 0 ? alpha : 0.0);
        vb[i] = v;
        hv[k * n + i] = v;
      }
      if (tid == 0) {
        hv[(n - 1) * n + k] = tau;
        eq[k] = (tau != 0.0) ? alpha : x0;  // T(k+1, k)
      }
      __syncthreads();
      if (tau != 0.0) {
        // p = tau A22 v
        for (int i = tid; i < m; i += kEvsThreads) {
          const double* row = A + (k + 1 + i) * lda + (k + 1);
          double acc = 0.0;
          for (int j = 0; j < m; ++j) acc += row[j] * vb[j];
          pb[i] = tau * acc;
        }
        __syncthreads();
        double vp = 0.0;
        for (int i = tid; i < m; i += kEvsThreads) vp += vb[i] * pb[i];
        const double K = 0.5 * tau * block_sum_256(vp, red);
        // w = p - K v
        for (int i = tid; i < m; i += kEvsThreads) pb[i] -= K * vb[i];
        __syncthreads();
        // A22 -= v w^T + w v^T
        for (int idx = tid; idx < m * m; idx += kEvsThreads) {
          const int i = idx / m, j = idx % m;
          A[(k + 1 + i) * lda + (k + 1 + j)] -= vb[i] * pb[j] + pb[i] * vb[j];
        }
      }
      __syncthreads();
    }
    for (int i = tid; i < n; i += kEvsThreads) dq[i] = A[i * lda + i];
    if (tid == 0) eq[n - 2] = A[(n - 1) * lda + (n - 2)];
    __syncthreads();
    // second copy of T for wave 1, Z = I
    for (int i = tid; i < n; i += kEvsThreads) {
      dq[n + i] = dq[i];
      eq[n + i] = (i < n - 1) ? eq[i] : 0.0;
      if (i == n - 1) eq[i] = 0.0;
    }
    for (int idx = tid; idx < n * n; idx += kEvsThreads) {
      const int i = idx / n, j = idx % n;
      A[i * lda + j] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    // ---- 2. implicit QL, waves 0 and 1, no barriers ----
    if (wave < 2) {
      double* d = dq + wave * n;
      double* e = eq + wave * n;
      const int row = wave * 64 + lane;
      double* z = A + min(row, n - 1) * lda;
      const bool own = row < n;
      const double eps = 2.220446049250313e-16;
      for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
          int m = l;
          while (m < n - 1 && !(fabs(e[m]) <= eps * (fabs(d[m]) + fabs(d[m + 1])))) ++m;
          if (m == l) break;
          if (iter >= 60) {
            if (lane == 0) bad = 1;
            break;
          }
          double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
          double r = hypot_scaled(g, 1.0);
          g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
          double sn = 1.0, cs = 1.0, pp = 0.0;
          bool deflated = false;
          for (int i = m - 1; i >= l; --i) {
            const double f = sn * e[i], b = cs * e[i];
            r = hypot_scaled(f, g);
            if (lane == 0) e[i + 1] = r;
            __builtin_amdgcn_wave_barrier();
            if (r == 0.0) {
              if (lane == 0) {
                d[i + 1] -= pp;
                e[m] = 0.0;
              }
              __builtin_amdgcn_wave_barrier();
              deflated = true;
              break;
            }
            sn = f / r;
            cs = g / r;
            g = d[i + 1] - pp;
            r = (d[i] - g) * sn + 2.0 * cs * b;
            pp = sn * r;
            if (lane == 0) d[i + 1] = g + pp;
            __builtin_amdgcn_wave_barrier();
            g = cs * r - b;
            if (own) {
              const double z1 = z[i + 1], z0 = z[i];
              z[i + 1] = sn * z0 + cs * z1;
              z[i] = cs * z0 - sn * z1;
            }
          }
          if (deflated) continue;
          if (lane == 0) {
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    __syncthreads();

    // ---- 3. small set, back-transformation of its columns, lumped diagonal ----
    double lm = -1e300;
    for (int i = tid; i < n; i += kEvsThreads) lm = fmax(lm, dq[i]);
    const double lmax = block_max_256(lm, red);
    double mg = 1e300;
    for (int i = tid; i < n; i += kEvsThreads) mg = fmin(mg, fabs(dq[i] / lmax - a.f_lambda));
    const double marg = -block_max_256(-mg, red);
    if (tid == 0) {
      int k = 0;
      for (int i = 0; i < n; ++i)
        if (dq[i] < a.f_lambda * lmax) cols[k++] = i;
      nsmall = k;
    }
    __syncthreads();
    const int ks = nsmall;
    for (int k = n - 3; k >= 0 && ks > 0; --k) {
      const int m = n - k - 1;
      for (int i = tid; i < m; i += kEvsThreads) vb[i] = hv[k * n + i];
      const double tau = hv[(n - 1) * n + k];
      __syncthreads();
      if (tau != 0.0) {
        for (int s = wave; s < ks; s += 4) {
          const int c = cols[s];
          double part = 0.0;
          for (int i = lane; i < m; i += 64) part += vb[i] * A[(k + 1 + i) * lda + c];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
          const double w = tau * part;
          for (int i = lane; i < m; i += 64) A[(k + 1 + i) * lda + c] -= vb[i] * w;
        }
      }
      __syncthreads();
    }
    double dmax = 0.0;
    for (int r = tid; r < n; r += kEvsThreads) {
      double acc = 0.0;
      for (int s = 0; s < ks; ++s) {
        const double x = A[r * lda + cols[s]];
        acc += x * x;
      }
      dk[r] = acc;
      dmax = fmax(dmax, acc);
    }
    const double maxd = block_max_256(dmax, red);
    for (int r = tid; r < n; r += kEvsThreads) {
      const double ms = (maxd > 0.0) ? (maxmf / maxd) * dk[r] : 0.0;
      a.lumped[q * n + r] = me / tr * dg[r] + a.eps * ms;
    }
    if (tid == 0) {
      a.margin[q] = marg;
      a.fail[q] = bad;
    }
    __syncthreads();
  }
}

fcw_status setup_stabilize(Ctx& c, double eps, double f_lambda) {
  if (c.n_cut_cand == 0) return FCW_OK;
  const int n = c.n_s;
  if (n > 256) {
    set_error("eigenvalue stabilisation supports at most 256 nodes per cell (got %d)", n);
    return FCW_E_UNSUPPORTED;
  }
  const int m = (n + 1) / 2 * 2;
  auto frame = [&](bool full) {
    size_t b = (size_t)(kEvsThreads + n + m) * sizeof(double) + (size_t)(m + 2) * sizeof(int);
    b = (b + 7) / 8 * 8;
    if (full) b += (size_t)2 * m * (m + 1) * sizeof(double);
    return b;
  };
  const size_t shbytes = frame(eps != 0.0);
  const int lda = (n % 2 == 1) ? n : n + 1;
  const size_t big_bytes = ((size_t)n * lda + kEvsThreads + 9 * (size_t)n) * sizeof(double) +
                           (size_t)n * sizeof(int);
  const bool big = shbytes > 160 * 1024;
  if (big && big_bytes > 160 * 1024) {
    set_error("eigenvalue stabilisation of n_s=%d does not fit in LDS", n);
    return FCW_E_UNSUPPORTED;
  }
  int32_t* fail = nullptr;
  FCW_HIP(hipMallocAsync((void**)&fail, c.n_cut_cand * 4, c.stream));
  if (big) {
    // one workgroup per CU, grid-stride over the cut cells; reflectors in scratch slots
    const int grid = (int)std::min<int64_t>(c.n_cut_cand, 256);
    double* scratch = nullptr;
    FCW_HIP(hipMallocAsync((void**)&scratch, (size_t)grid * n * n * sizeof(double), c.stream));
    EvsBigArgs eb{};
    eb.n = n;
    eb.lda = lda;
    eb.mcut = c.d_mcut;
    eb.mfull = c.d_mfull;
    eb.eps = eps;
    eb.f_lambda = f_lambda;
    eb.ncand = c.n_cut_cand;
    eb.scratch = scratch;
    eb.lumped = c.d_lumped;
    eb.margin = c.d_margin;
    eb.fail = fail;
    FCW_HIP(hipFuncSetAttribute((const void*)evs_big_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)big_bytes));
    evs_big_kernel<<<grid, kEvsThreads, big_bytes, c.stream>>>(eb);
    FCW_HIP(hipGetLastError());
    FCW_HIP(hipFreeAsync(scratch, c.stream));
  }
  EvsArgs ea{};
  ea.n = n;
  ea.m = m;
  ea.mcut = c.d_mcut;
  ea.mfull = c.d_mfull;
  ea.eps = eps;
  ea.f_lambda = f_lambda;
  ea.max_sweeps = 60;
  ea.tol = 1e-14;
  ea.tol_abs = 1e-17;
  ea.lumped = c.d_lumped;
  ea.margin = c.d_margin;
  ea.fail = fail;
  if (!big) {
    FCW_HIP(hipFuncSetAttribute((const void*)evs_lump_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shbytes));
    evs_lump_kernel<<<(unsigned)c.n_cut_cand, kEvsThreads, shbytes, c.stream>>>(ea);
    FCW_HIP(hipGetLastError());
  }
  std::vector<int32_t> hf(c.n_cut_cand), hav(c.n_cut_cand);
  FCW_HIP(hipMemcpyAsync(hf.data(), fail, c.n_cut_cand * 4, hipMemcpyDeviceToHost, c.stream));
  FCW_HIP(hipMemcpyAsync(hav.data(), c.d_all_void, c.n_cut_cand * 4, hipMemcpyDeviceToHost,
                         c.stream));
  FCW_HIP(hipFreeAsync(fail, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  for (int64_t i = 0; i < c.n_cut_cand; ++i) {
    if (hf[i] && !hav[i]) {
      set_error("eigenvalue stabilisation did not converge in cut cell %lld",
                (long long)i);
      return FCW_E_NOCONV;
    }
  }
  return FCW_OK;
}

// --------------------------------------------------------------------------------
// Reclassification, mass assembly, packing
// --------------------------------------------------------------------------------

__global__ void reclassify_kernel(const int32_t* cut_cells, const int32_t* all_void, int64_t n,
                                  int8_t* cls, int32_t* info) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  if (all_void[q]) {
    int cell = cut_cells[q];
    cls[cell] = kClsOut;
    info[cell] = kInfoOut;
  }
}

struct MassArgs {
  int dim, p;
  int n[3], np[3];
  int64_t nnodes;
  const int32_t* info;
  const double* lref;
  const double* lumped;
  double* mass;
  double* invm64;
};

// diagonal mass per node: sum of the lumped element diagonals of the active cells
// around it, adjacent cells taken in lexicographic order (z, y, x; lower first)
__global__ void mass_kernel(MassArgs a) {
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= a.nnodes) return;
  int idx[3] = {0, 0, 0};
  int64_t r = node;
  for (int k = 0; k < a.dim; ++k) { idx[k] = (int)(r % a.np[k]); r /= a.np[k]; }
  int cl[3], ch[3];
  for (int k = 0; k < 3; ++k) {
    if (k >= a.dim) { cl[k] = ch[k] = 0; continue; }
    int i = idx[k];
    int hi = i / a.p;
    int lo = (i % a.p == 0) ? hi - 1 : hi;
    if (hi > a.n[k] - 1) hi = a.n[k] - 1;
    if (lo < 0) lo = 0;
    cl[k] = lo;
    ch[k] = hi;
  }
  const int np1 = a.p + 1;
  int ns = 1;
  for (int k = 0; k < a.dim; ++k) ns *= np1;
  double m = 0.0;
  for (int cz = cl[2]; cz <= ch[2]; ++cz)
    for (int cy = cl[1]; cy <= ch[1]; ++cy)
      for (int cx = cl[0]; cx <= ch[0]; ++cx) {
        int64_t cell = cx + (int64_t)a.n[0] * (cy + (int64_t)a.n[1] * cz);
        int inf = a.info[cell];
        if (inf == kInfoOut) continue;
        int loc = (idx[0] - cx * a.p);
        if (a.dim > 1) loc += np1 * (idx[1] - cy * a.p);
        if (a.dim > 2) loc += np1 * np1 * (idx[2] - cz * a.p);
        m += (inf == kInfoUncut) ? a.lref[loc] : a.lumped[(int64_t)inf * ns + loc];
      }
  a.mass[node] = m;
  a.invm64[node] = (m > 0.0) ? 1.0 / m : 0.0;
}

// 1-D inverse assembled GLL weights per direction: node g of direction k collects
// w[g % p] inside a cell, w[p] + w[0] where two cells meet, one of them at the box faces
__global__ void invw_kernel(const RefTables* tab, int dim, int p, int n0, int n1, int n2,
                            double* invw) {
  const int np[3] = {n0 * p + 1, n1 * p + 1, n2 * p + 1};
  const int n[3] = {n0, n1, n2};
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  int off = 0;
  for (int k = 0; k < dim; ++k) {
    if (g < np[k]) {
      const int r = g % p;
      double w;
      if (r != 0) w = tab->gll_w[r];
      else w = (g > 0 ? tab->gll_w[p] : 0.0) + (g < n[k] * p ? tab->gll_w[0] : 0.0);
      invw[off + g] = 1.0 / w;
      return;
    }
    g -= np[k];
    off += np[k];
  }
}

// per node: does its mass differ from the analytic uncut value (a cell around it is cut
// or outside)?  Then the stored inverse is the assembled one, else the analytic one.
struct InvmArgs {
  int dim, p;
  int n[3], np[3];
  int64_t nnodes;
  const int32_t* info;
  const double* invm64;
  const double* invw;
  double cm;
  int8_t* needs;
};

template <typename T>
__global__ void invm_kernel(InvmArgs a, T* out) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= a.nnodes) return;
  int idx[3] = {0, 0, 0};
  int64_t r = node;
  for (int k = 0; k < a.dim; ++k) { idx[k] = (int)(r % a.np[k]); r /= a.np[k]; }
  int cl[3] = {0, 0, 0}, ch[3] = {0, 0, 0};
  for (int k = 0; k < a.dim; ++k) {
    const int i = idx[k];
    int hi = i / a.p;
    int lo = (i % a.p == 0) ? hi - 1 : hi;
    cl[k] = max(lo, 0);
    ch[k] = min(hi, a.n[k] - 1);
  }
  bool needs = false;
  for (int cz = cl[2]; cz <= ch[2]; ++cz)
    for (int cy = cl[1]; cy <= ch[1]; ++cy)
      for (int cx = cl[0]; cx <= ch[0]; ++cx)
        if (a.info[cx + (int64_t)a.n[0] * (cy + (int64_t)a.n[1] * cz)] != kInfoUncut) needs = true;
  a.needs[node] = needs ? 1 : 0;
  const double iy = (a.dim > 1) ? a.invw[a.np[0] + idx[1]] : 1.0;
  const double iz = (a.dim > 2) ? a.invw[a.np[0] + a.np[1] + idx[2]] : 1.0;
  out[node] = needs ? (T)a.invm64[node] : analytic_invm<T>(a.cm, a.invw[idx[0]], iy, iz);
}

// bit b of word w of node row R: node (32 w + b) of that row needs the stored inverse
__global__ void mflag_kernel(const int8_t* needs, uint32_t* words, int npx, int64_t nrows,
                             int wpr) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nrows * wpr) return;
  const int64_t row = w / wpr;
  const int wi = (int)(w % wpr);
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const int gx = wi * 32 + b;
    if (gx < npx && needs[row * npx + gx]) bits |= 1u << b;
  }
  words[w] = bits;
}

// FP64 -> bf16, rounded to nearest even directly from the double (no FP32 double
// rounding); finite normal inputs in the FP32 exponent range, and zero
__device__ static uint16_t bf16_rne(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
  const int e = (int)((b >> 52) & 0x7ff);
  if (e == 0) return sign;
  if (e < 1023 - 126 || e > 1023 + 127) {  // outside the normal range: through FP32
    const uint32_t f = __float_as_uint((float)x);
    return (uint16_t)((f + 0x7fffu + ((f >> 16) & 1u)) >> 16);
  }
  const uint64_t m = b & ((1ull << 52) - 1);
  uint32_t v = (uint32_t)((e - 1023 + 127) << 7) | (uint32_t)(m >> 45);
  const uint64_t rest = m & ((1ull << 45) - 1), half = 1ull << 44;
  if (rest > half || (rest == half && (v & 1u))) ++v;  // a carry moves into the exponent
  return (uint16_t)(sign | (v & 0x7fffu));
}

__device__ static double bf16_value(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

// K_ref split into bf16 hi + lo (hi = nearest bf16 of K, lo = nearest bf16 of K - hi),
// laid out as the MFMA A fragments of 16x16x32: [mb][kb][hi/lo][lane][e] holds row
// mb*16 + lane%16, column kb*32 + 8*(lane/16) + e (zero outside the matrix)
__global__ void bf16_frag_kernel(const double* k, uint16_t* out, int nl, int nmb, int nkb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nmb * nkb * 64 * 8;
  if (t >= total) return;
  const int e = (int)(t % 8), lane = (int)((t / 8) % 64);
  const int kb = (int)((t / 512) % nkb), mb = (int)(t / (512 * nkb));
  const int r = mb * 16 + lane % 16, cc = kb * 32 + 8 * (lane / 16) + e;
  const double v = (r < nl && cc < nl) ? k[(int64_t)r * nl + cc] : 0.0;
  const uint16_t hi = bf16_rne(v);
  const uint16_t lo = bf16_rne(v - bf16_value(hi));
  const int64_t base = (((int64_t)mb * nkb + kb) * 2) * 64 * 8 + lane * 8 + e;
  out[base] = hi;
  out[base + 64 * 8] = lo;
}

template <typename T>
__global__ void cast_kernel(const double* in, T* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

// packed upper triangle, column-major: entry (i, j), i <= j, at j (j + 1) / 2 + i
template <typename T>
__global__ void pack_upper_kernel(const double* k, T* out, int nl, int64_t ncut) {
  const int64_t np = (int64_t)nl * (nl + 1) / 2;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= np * ncut) return;
  int64_t q = g / np;
  int lin = (int)(g % np);
  int j = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= lin) ++j;
  while (j * (j + 1) / 2 > lin) --j;
  int i = lin - j * (j + 1) / 2;
  out[g] = (T)k[q * nl * nl + (int64_t)i * nl + j];
}

fcw_status setup_reclassify(Ctx& c) {
  if (c.n_cut_cand > 0) {
    reclassify_kernel<<<(unsigned)((c.n_cut_cand + 255) / 256), 256, 0, c.stream>>>(
        c.d_cut_cells, c.d_all_void, c.n_cut_cand, c.d_cls, c.d_info);
    FCW_HIP(hipGetLastError());
  }
  std::vector<int8_t> cls(c.ncell_total);
  FCW_HIP(hipMemcpyAsync(cls.data(), c.d_cls, cls.size(), hipMemcpyDeviceToHost, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  int64_t cnt[3] = {0, 0, 0};
  for (int8_t k : cls) cnt[k]++;
  c.n_out = cnt[kClsOut];
  c.n_uncut = cnt[kClsUncut];
  c.n_cut = cnt[kClsCut];
  return FCW_OK;
}

fcw_status setup_mass_and_pack(Ctx& c) {
  MassArgs ma{};
  ma.dim = c.dim;
  ma.p = c.p;
  for (int k = 0; k < 3; ++k) { ma.n[k] = c.ncells[k]; ma.np[k] = c.npts[k]; }
  ma.nnodes = c.nnodes;
  ma.info = c.d_info;
  ma.lref = c.d_lref;
  ma.lumped = c.d_lumped;
  ma.mass = c.d_mass;
  ma.invm64 = c.d_invm64;
  mass_kernel<<<(unsigned)((c.nnodes + 255) / 256), 256, 0, c.stream>>>(ma);
  FCW_HIP(hipGetLastError());
  const int64_t nl = c.n_loc;
  const int64_t npk = nl * (nl + 1) / 2;
  const unsigned gn = (unsigned)((c.nnodes + 255) / 256);
  const unsigned gk = (unsigned)((nl * nl + 255) / 256);
  const unsigned gp = (unsigned)((npk * c.n_cut_cand + 255) / 256);
  // analytic inverse masses and the per-node flags
  const int npsum = c.npts[0] + (c.dim > 1 ? c.npts[1] : 0) + (c.dim > 2 ? c.npts[2] : 0);
  const int64_t nrows = c.nnodes / c.npts[0];
  c.mflag_wpr = (c.npts[0] + 31) / 32 + 6;  // room for the words a kernel row read spans
  if (!c.d_invw) {
    FCW_HIP(hipMalloc((void**)&c.d_invw, (size_t)npsum * sizeof(double)));
    FCW_HIP(hipMalloc((void**)&c.d_mflag, (size_t)nrows * c.mflag_wpr * sizeof(uint32_t)));
    c.footprint += (int64_t)npsum * 8 + nrows * c.mflag_wpr * 4;
  }
  {
    double m = c.rho;
    for (int k = 0; k < c.dim; ++k) m *= 0.5 * c.h;
    c.cm = 1.0 / m;
  }
  invw_kernel<<<(npsum + 255) / 256, 256, 0, c.stream>>>(c.d_tab, c.dim, c.p, c.ncells[0],
                                                        c.dim > 1 ? c.ncells[1] : 1,
                                                        c.dim > 2 ? c.ncells[2] : 1, c.d_invw);
  FCW_HIP(hipGetLastError());
  int8_t* needs = nullptr;
  FCW_HIP(hipMallocAsync((void**)&needs, c.nnodes, c.stream));
  InvmArgs ia{};
  ia.dim = c.dim;
  ia.p = c.p;
  for (int k = 0; k < 3; ++k) { ia.n[k] = c.ncells[k]; ia.np[k] = c.npts[k]; }
  ia.nnodes = c.nnodes;
  ia.info = c.d_info;
  ia.invm64 = c.d_invm64;
  ia.invw = c.d_invw;
  ia.cm = c.cm;
  ia.needs = needs;
  if (c.precision == FCW_FP64) {
    invm_kernel<double><<<gn, 256, 0, c.stream>>>(ia, (double*)c.d_invm);
    cast_kernel<double><<<gk, 256, 0, c.stream>>>(c.d_kref, (double*)c.d_kref_s, nl * nl);
    if (c.n_cut_cand > 0)
      pack_upper_kernel<double><<<gp, 256, 0, c.stream>>>(c.d_kcut, (double*)c.d_kcut_s, (int)nl,
                                                          c.n_cut_cand);
  } else {
    if (c.precision == FCW_BF16) {
      const int nmb = (int)((nl + 15) / 16), nkb = (int)((nl + 31) / 32);
      const int64_t nfrag = (int64_t)nmb * nkb * 2 * 64 * 8;  // bf16 values
      if (!c.d_kref_bf) {
        FCW_HIP(hipMalloc(&c.d_kref_bf, (size_t)nfrag * 2));
        c.footprint += nfrag * 2;
      }
      bf16_frag_kernel<<<(unsigned)((nfrag / 2 + 255) / 256), 256, 0, c.stream>>>(
          c.d_kref, (uint16_t*)c.d_kref_bf, (int)nl, nmb, nkb);
    }
    invm_kernel<float><<<gn, 256, 0, c.stream>>>(ia, (float*)c.d_invm);
    cast_kernel<float><<<gk, 256, 0, c.stream>>>(c.d_kref, (float*)c.d_kref_s, nl * nl);
    if (c.n_cut_cand > 0)
      pack_upper_kernel<float><<<gp, 256, 0, c.stream>>>(c.d_kcut, (float*)c.d_kcut_s, (int)nl,
                                                         c.n_cut_cand);
  }
  FCW_HIP(hipGetLastError());
  const int64_t nw = nrows * c.mflag_wpr;
  mflag_kernel<<<(unsigned)((nw + 255) / 256), 256, 0, c.stream>>>(needs, c.d_mflag, c.npts[0],
                                                                   nrows, c.mflag_wpr);
  FCW_HIP(hipGetLastError());
  FCW_HIP(hipFreeAsync(needs, c.stream));
  return FCW_OK;
}

// --------------------------------------------------------------------------------
// Point-source load vectors
// --------------------------------------------------------------------------------

struct SrcArgs {
  Grid g;
  int p, ncomp;
  double rho;
  const RefTables* tab;
  int nsrc;
  const fcw_source* in;
  SourceDev* out;
};

template <int NP1>
__global__ void source_kernel(SrcArgs a) {
#pragma clang fp contract(off)
  const int s = blockIdx.x;
  if (s >= a.nsrc || threadIdx.x != 0) return;
  const fcw_source& in = a.in[s];
  SourceDev& o = a.out[s];
  double L[3][NP1], dL[3][NP1];
  for (int k = 0; k < 3; ++k) o.cell[k] = 0;
  for (int k = 0; k < a.g.dim; ++k) {
    int i = (int)floor((in.x[k] - a.g.lo[k]) / a.g.h);
    i = max(0, min(i, a.g.n[k] - 1));
    o.cell[k] = i;
    double clo = a.g.lo[k] + (double)i * a.g.h;
    double xi = 2.0 * (in.x[k] - clo) / a.g.h - 1.0;
    lagrange_1d<NP1>(a.tab->gll_x, xi, L[k], dL[k]);
  }
  int ns = 1;
  for (int k = 0; k < a.g.dim; ++k) ns *= NP1;
  for (int loc = 0; loc < ns; ++loc) {
    double N = 1.0;
    int r = loc;
    for (int k = 0; k < a.g.dim; ++k) { N *= L[k][r % NP1]; r /= NP1; }
    for (int cc = 0; cc < a.ncomp; ++cc) {
      double dc = (a.ncomp == 1) ? 1.0 : in.dir[cc];
      o.b[cc * ns + loc] = (in.sigma > 0.0) ? 0.0 : a.rho * in.amp * dc * N;
    }
  }
  // a volumetric source has no point load: its cell lies far outside every tile
  if (in.sigma > 0.0)
    for (int k = 0; k < 3; ++k) o.cell[k] = -(1 << 20);
  o.f0 = in.f0;
}

// --------------------------------------------------------------------------------
// Volumetric Gaussian sources (Sec. 3.1)
// --------------------------------------------------------------------------------

struct GaussArgs {
  Grid g;
  CubeGeo cube;
  int nvoids;
  const double* vc;
  const double* vr;
  double alpha, rho;
  const RefTables* tab;
  const int32_t* cells;  // support cells
  int ncell;
  double xs[3], sigma, amp;
  int m;                 // boxes per direction in a cell
  double* y;             // [ncell][n_s]: rho amp int alpha^FCM g N_a over the cell
};

// y[e][a] = rho amp int_cell alpha^FCM(x) exp(-|x - x_s|^2 / (2 sigma^2)) N_a(x) dx with
// m^dim boxes and a Gauss-Legendre rule of NP1 + 2 = p + 3 points per direction on each;
// one block per support cell, thread a sums its shape function's terms in point order.
template <int NP1>
__global__ __launch_bounds__(128) void gauss_cells_kernel(GaussArgs a) {
#pragma clang fp contract(off)
  constexpr int NQ = NP1 + 2;
  __shared__ double qx[NQ], qw[NQ];
  if (threadIdx.x == 0) gl_rule(NQ, qx, qw);
  __syncthreads();
  const int dim = a.g.dim;
  const int ns = (dim == 3) ? NP1 * NP1 * NP1 : NP1 * NP1;
  const int la = threadIdx.x;
  if (la >= ns || blockIdx.x >= (unsigned)a.ncell) return;
  int ai[3] = {la % NP1, (la / NP1) % NP1, la / (NP1 * NP1)};
  double lo[3], hi[3];
  cell_box(a.g, a.cells[blockIdx.x], lo, hi);
  const double sub = a.g.h / a.m;
  const int nbox = (dim == 3) ? a.m * a.m * a.m : a.m * a.m;
  const int nq = (dim == 3) ? NQ * NQ * NQ : NQ * NQ;
  const double* gll = a.tab->gll_x;
  double acc = 0.0;
  for (int b = 0; b < nbox; ++b) {
    const int bi[3] = {b % a.m, (b / a.m) % a.m, b / (a.m * a.m)};
    for (int q = 0; q < nq; ++q) {
      const int qi[3] = {q % NQ, (q / NQ) % NQ, q / (NQ * NQ)};
      double x[3], w = 1.0, r2 = 0.0, N = 1.0;
      for (int k = 0; k < dim; ++k) {
        const double blo = lo[k] + sub * (double)bi[k];
        x[k] = blo + 0.5 * sub * (qx[qi[k]] + 1.0);
        w = w * (qw[qi[k]] * (0.5 * sub));
        r2 = r2 + (x[k] - a.xs[k]) * (x[k] - a.xs[k]);
        // Lagrange polynomial a_k on the GLL nodes at the local coordinate of x
        const double xi = 2.0 * (x[k] - lo[k]) / a.g.h - 1.0;
        double l = 1.0;
        for (int j = 0; j < NP1; ++j)
          if (j != ai[k]) l *= (xi - gll[j]) / (gll[ai[k]] - gll[j]);
        N = N * l;
      }
      bool fict = a.cube.on && cube_point_outside(a.cube, x);
      for (int v = 0; v < a.nvoids && !fict; ++v) {
        const double* c = a.vc + (int64_t)v * dim;
        double d2 = 0.0;
        for (int k = 0; k < dim; ++k) d2 = d2 + (x[k] - c[k]) * (x[k] - c[k]);
        fict = d2 < a.vr[v] * a.vr[v];
      }
      const double al = fict ? a.alpha : 1.0;
      const double gv = exp(-0.5 * r2 / (a.sigma * a.sigma));
      acc = acc + ((w * al) * gv) * N;
    }
  }
  a.y[(int64_t)blockIdx.x * ns + la] = a.rho * a.amp * acc;
}

// b over the support nodes: node k sums its (cell slot, local node) entries in order;
// every component gets dir_c times it
__global__ void gauss_gather_kernel(const double* y, int ns, const int32_t* eoff,
                                    const int32_t* ent, const int64_t* node, int nnode,
                                    int ncomp, double d0, double d1, double d2, int64_t nnodes,
                                    int64_t* dof_out, double* val_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnode) return;
  double b = 0.0;
  for (int e = eoff[k]; e < eoff[k + 1]; ++e) b = b + y[ent[e]];
  const double dir[3] = {d0, d1, d2};
  for (int c = 0; c < ncomp; ++c) {
    dof_out[(int64_t)c * nnode + k] = (int64_t)c * nnodes + node[k];
    val_out[(int64_t)c * nnode + k] = (ncomp == 1) ? b : dir[c] * b;
  }
}

// Load vectors of the volumetric sources among src[0..nrhs): entries [g_off[r], g_off[r+1])
// of d_gdof / d_gval for right-hand side r (empty for point sources).
static fcw_status prepare_gauss(Ctx& c, int nrhs, const fcw_source* src) {
  c.g_off.assign(nrhs + 1, 0);
  c.g_active = false;
  bool any = false;
  for (int r = 0; r < nrhs; ++r) any = any || src[r].sigma > 0.0;
  if (!any) return FCW_OK;
  if (c.h_cls.empty()) {
    c.h_cls.resize(c.ncell_total);
    FCW_HIP(hipMemcpyAsync(c.h_cls.data(), c.d_cls, c.ncell_total, hipMemcpyDeviceToHost,
                           c.stream));
    FCW_HIP(hipStreamSynchronize(c.stream));
  }
  const int ns = c.n_s, np1 = c.p + 1;
  // host bookkeeping per source: support cells, their nodes and the gather lists
  struct Part {
    std::vector<int32_t> cells, eoff, ent;
    std::vector<int64_t> node;
  };
  std::vector<Part> parts(nrhs);
  int64_t total = 0;
  for (int r = 0; r < nrhs; ++r) {
    if (!(src[r].sigma > 0.0)) continue;
    Part& pt = parts[r];
    const double sg = src[r].sigma;
    int ilo[3] = {0, 0, 0}, ihi[3] = {1, 1, 1};
    for (int k = 0; k < c.dim; ++k) {
      ilo[k] = std::max(0, (int)std::floor((src[r].x[k] - 8.0 * sg - c.lo[k]) / c.h) - 1);
      ihi[k] = std::min(c.ncells[k], (int)std::floor((src[r].x[k] + 8.0 * sg - c.lo[k]) / c.h) + 2);
    }
    for (int iz = ilo[2]; iz < ihi[2]; ++iz)
      for (int iy = ilo[1]; iy < ihi[1]; ++iy)
        for (int ix = ilo[0]; ix < ihi[0]; ++ix) {
          const int64_t cell = ix + (int64_t)c.ncells[0] * (iy + (int64_t)c.ncells[1] * iz);
          if (c.h_cls[cell] == kClsOut) continue;
          const int idx[3] = {ix, iy, iz};
          double d2 = 0.0;
          for (int k = 0; k < c.dim; ++k) {
            const double blo = c.lo[k] + (double)idx[k] * c.h;
            const double bhi = c.lo[k] + (double)(idx[k] + 1) * c.h;
            const double gap = std::max(std::max(blo - src[r].x[k], 0.0), src[r].x[k] - bhi);
            d2 = d2 + gap * gap;
          }
          if (d2 < 64.0 * sg * sg) pt.cells.push_back((int32_t)cell);
        }
    // the cells above come in increasing cell order (x fastest); their nodes, and per
    // node the (slot, local node) entries in slot order
    std::vector<std::pair<int64_t, int32_t>> pairs;  // (node, slot * ns + a)
    for (size_t q = 0; q < pt.cells.size(); ++q) {
      const int64_t cell = pt.cells[q];
      const int64_t cx = cell % c.ncells[0], cy = (cell / c.ncells[0]) % c.ncells[1],
                    cz = cell / ((int64_t)c.ncells[0] * c.ncells[1]);
      for (int a = 0; a < ns; ++a) {
        const int ax = a % np1, ay = (a / np1) % np1, az = a / (np1 * np1);
        const int64_t gx = cx * c.p + ax, gy = cy * c.p + ay, gz = (c.dim == 3) ? cz * c.p + az : 0;
        const int64_t nd = gx + (int64_t)c.npts[0] * (gy + (int64_t)c.npts[1] * gz);
        pairs.emplace_back(nd, (int32_t)(q * ns + a));
      }
    }
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                       return x.first < y.first;
                     });
    for (size_t i = 0; i < pairs.size(); ++i) {
      if (i == 0 || pairs[i].first != pairs[i - 1].first) {
        pt.node.push_back(pairs[i].first);
        pt.eoff.push_back((int32_t)pt.ent.size());
      }
      pt.ent.push_back(pairs[i].second);
    }
    pt.eoff.push_back((int32_t)pt.ent.size());
    total += (int64_t)pt.node.size() * c.ncomp;
  }
  for (int r = 0; r < nrhs; ++r)
    c.g_off[r + 1] = c.g_off[r] + (int32_t)(parts[r].node.size() * c.ncomp);
  if ((size_t)total > c.g_cap) {
    if (c.d_gdof) FCW_HIP(hipFree(c.d_gdof));
    if (c.d_gval) FCW_HIP(hipFree(c.d_gval));
    c.d_gdof = nullptr;
    c.d_gval = nullptr;
    c.footprint -= (int64_t)c.g_cap * 16;
    FCW_HIP(hipMalloc((void**)&c.d_gdof, total * sizeof(int64_t)));
    FCW_HIP(hipMalloc((void**)&c.d_gval, total * sizeof(double)));
    c.g_cap = (size_t)total;
    c.footprint += (int64_t)c.g_cap * 16;
  }
  if (!c.d_goff) {
    FCW_HIP(hipMalloc((void**)&c.d_goff, (kMaxSrc + 1) * sizeof(int32_t)));
    c.footprint += (kMaxSrc + 1) * sizeof(int32_t);
  }
  FCW_HIP(hipMemcpyAsync(c.d_goff, c.g_off.data(), (nrhs + 1) * sizeof(int32_t),
                         hipMemcpyHostToDevice, c.stream));
  for (int r = 0; r < nrhs; ++r) {
    Part& pt = parts[r];
    if (pt.cells.empty()) continue;
    const int nc = (int)pt.cells.size(), nn = (int)pt.node.size();
    int32_t *dcells = nullptr, *deoff = nullptr, *dent = nullptr;
    int64_t* dnode = nullptr;
    double* dy = nullptr;
    auto release = [&]() {
      if (dcells) (void)hipFree(dcells);
      if (deoff) (void)hipFree(deoff);
      if (dent) (void)hipFree(dent);
      if (dnode) (void)hipFree(dnode);
      if (dy) (void)hipFree(dy);
    };
    hipError_t e = hipMalloc((void**)&dcells, nc * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&deoff, (nn + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&dent, pt.ent.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&dnode, nn * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&dy, (size_t)nc * ns * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpyAsync(dcells, pt.cells.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(deoff, pt.eoff.data(), (nn + 1) * sizeof(int32_t), hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dent, pt.ent.data(), pt.ent.size() * sizeof(int32_t), hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dnode, pt.node.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) {
      release();
      return hip_fail(e, "volumetric source staging");
    }
    GaussArgs ga{};
    ga.g = make_grid(c);
    ga.cube = c.cube;
    ga.nvoids = c.nvoids;
    ga.vc = c.d_void_c;
    ga.vr = c.d_void_r;
    ga.alpha = c.alpha;
    ga.rho = c.rho;
    ga.tab = c.d_tab;
    ga.cells = dcells;
    ga.ncell = nc;
    for (int k = 0; k < 3; ++k) ga.xs[k] = src[r].x[k];
    ga.sigma = src[r].sigma;
    ga.amp = src[r].amp;
    ga.m = std::max(1, std::min(64, (int)std::ceil(c.h / src[r].sigma)));
    ga.y = dy;
    switch (np1) {
      case 2: gauss_cells_kernel<2><<<nc, 128, 0, c.stream>>>(ga); break;
      case 3: gauss_cells_kernel<3><<<nc, 128, 0, c.stream>>>(ga); break;
      case 4: gauss_cells_kernel<4><<<nc, 128, 0, c.stream>>>(ga); break;
      case 5: gauss_cells_kernel<5><<<nc, 128, 0, c.stream>>>(ga); break;
      default:
        release();
        set_error("volumetric sources not built for p=%d", c.p);
        return FCW_E_UNSUPPORTED;
    }
    gauss_gather_kernel<<<(nn + 255) / 256, 256, 0, c.stream>>>(
        dy, ns, deoff, dent, dnode, nn, c.ncomp, src[r].dir[0], src[r].dir[1], src[r].dir[2],
        c.nnodes, c.d_gdof + c.g_off[r], c.d_gval + c.g_off[r]);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    release();
    if (e != hipSuccess) return hip_fail(e, "volumetric source integration");
  }
  c.g_active = true;
  return FCW_OK;
}

// Receivers: the cell holding each point (the rule of the sources) and N_a(x_r).
struct RecArgs {
  Grid g;
  const RefTables* tab;
  int nrec;
  const double* x;  // [nrec][3]
  RecDev* out;
};

template <int NP1>
__global__ void receiver_kernel(RecArgs a) {
#pragma clang fp contract(off)
  const int r = blockIdx.x;
  if (r >= a.nrec || threadIdx.x != 0) return;
  const double* x = a.x + 3 * r;
  RecDev& o = a.out[r];
  double L[3][NP1], dL[3][NP1];
  for (int k = 0; k < 3; ++k) o.cell[k] = 0;
  for (int k = 0; k < a.g.dim; ++k) {
    int i = (int)floor((x[k] - a.g.lo[k]) / a.g.h);
    i = max(0, min(i, a.g.n[k] - 1));
    o.cell[k] = i;
    const double clo = a.g.lo[k] + (double)i * a.g.h;
    const double xi = 2.0 * (x[k] - clo) / a.g.h - 1.0;
    lagrange_1d<NP1>(a.tab->gll_x, xi, L[k], dL[k]);
  }
  int ns = 1;
  for (int k = 0; k < a.g.dim; ++k) ns *= NP1;
  for (int loc = 0; loc < ns; ++loc) {
    double N = 1.0;
    int q = loc;
    for (int k = 0; k < a.g.dim; ++k) { N *= L[k][q % NP1]; q /= NP1; }
    o.w[loc] = N;
  }
}

fcw_status prepare_receivers(Ctx& c, int nrec, const double* x) {
  if (nrec <= 0) return FCW_OK;
  if (nrec > FCW_MAX_RECEIVERS) {
    set_error("at most %d receivers per problem (got %d)", FCW_MAX_RECEIVERS, nrec);
    return FCW_E_ARG;
  }
  if (!c.d_rec) {
    // RecDev[FCW_MAX_RECEIVERS] followed by a staging copy of the points
    FCW_HIP(hipMalloc((void**)&c.d_rec,
                      FCW_MAX_RECEIVERS * (sizeof(RecDev) + 3 * sizeof(double))));
    c.footprint += FCW_MAX_RECEIVERS * (sizeof(RecDev) + 3 * sizeof(double));
  }
  double* staged = (double*)(c.d_rec + FCW_MAX_RECEIVERS);
  FCW_HIP(hipMemcpyAsync(staged, x, (size_t)nrec * 3 * sizeof(double), hipMemcpyHostToDevice,
                         c.stream));
  RecArgs ra{};
  ra.g = make_grid(c);
  ra.tab = c.d_tab;
  ra.nrec = nrec;
  ra.x = staged;
  ra.out = c.d_rec;
  switch (c.p + 1) {
    case 2: receiver_kernel<2><<<nrec, 64, 0, c.stream>>>(ra); break;
    case 3: receiver_kernel<3><<<nrec, 64, 0, c.stream>>>(ra); break;
    case 4: receiver_kernel<4><<<nrec, 64, 0, c.stream>>>(ra); break;
    case 5: receiver_kernel<5><<<nrec, 64, 0, c.stream>>>(ra); break;
    case 6: receiver_kernel<6><<<nrec, 64, 0, c.stream>>>(ra); break;
    case 7: receiver_kernel<7><<<nrec, 64, 0, c.stream>>>(ra); break;
    default:
      set_error("receivers not built for p=%d", c.p);
      return FCW_E_UNSUPPORTED;
  }
  FCW_HIP(hipGetLastError());
  // the host points must stay valid until the copy has run
  FCW_HIP(hipStreamSynchronize(c.stream));
  return FCW_OK;
}

fcw_status prepare_sources(Ctx& c, int nrhs, const fcw_source* src, bool remember) {
  if (nrhs > kMaxSrc) {
    set_error("at most %d right-hand sides per call (got %d)", kMaxSrc, nrhs);
    return FCW_E_ARG;
  }
  if (!remember)
    for (int r = 0; r < nrhs; ++r)
      if (src[r].sigma > 0.0) {
        set_error("volumetric sources need fcw_step_explicit or fcw_run (source %d)", r);
        return FCW_E_ARG;
      }
  if (!c.d_src) {
    // SourceDev[kMaxSrc] followed by a staging copy of the caller's fcw_source[kMaxSrc]
    FCW_HIP(hipMalloc((void**)&c.d_src, kMaxSrc * (sizeof(SourceDev) + sizeof(fcw_source))));
    c.src_cap = kMaxSrc;
    c.footprint += kMaxSrc * (sizeof(SourceDev) + sizeof(fcw_source));
  }
  // unchanged sources (the usual case for a run split into several calls) are kept
  if (remember && (int)c.src_staged.size() == nrhs &&
      std::memcmp(c.src_staged.data(), src, nrhs * sizeof(fcw_source)) == 0)
    return FCW_OK;
  c.src_staged.clear();
  fcw_source* staged = (fcw_source*)(c.d_src + kMaxSrc);
  FCW_HIP(hipMemcpyAsync(staged, src, nrhs * sizeof(fcw_source), hipMemcpyHostToDevice,
                         c.stream));
  SrcArgs sa{};
  sa.g = make_grid(c);
  sa.p = c.p;
  sa.ncomp = c.ncomp;
  sa.rho = c.rho;
  sa.tab = c.d_tab;
  sa.nsrc = nrhs;
  sa.in = staged;
  sa.out = c.d_src;
  switch (c.p + 1) {
    case 2: source_kernel<2><<<nrhs, 64, 0, c.stream>>>(sa); break;
    case 3: source_kernel<3><<<nrhs, 64, 0, c.stream>>>(sa); break;
    case 4: source_kernel<4><<<nrhs, 64, 0, c.stream>>>(sa); break;
    case 5: source_kernel<5><<<nrhs, 64, 0, c.stream>>>(sa); break;
    case 6: source_kernel<6><<<nrhs, 64, 0, c.stream>>>(sa); break;
    case 7: source_kernel<7><<<nrhs, 64, 0, c.stream>>>(sa); break;
    default:
      set_error("sources not built for p=%d", c.p);
      return FCW_E_UNSUPPORTED;
  }
  FCW_HIP(hipGetLastError());
  // the staged host array must stay valid until the copy has run
  FCW_HIP(hipStreamSynchronize(c.stream));
  if (!remember) return FCW_OK;  // (volumetric sources were refused above)
  fcw_status st = prepare_gauss(c, nrhs, src);
  if (st) {
    c.src_staged.clear();
    return st;
  }
  c.src_staged.assign(src, src + nrhs);
  return FCW_OK;
}

}  // namespace fcw
