// IGA-FCM on the device: the immersed scalar wave problem discretised with B-splines
// (paper Sec. 2.2: B-spline shape functions, the isogeometric variant of the finite cell
// method; Sec. 2.4: row-sum lumping; Table methods: IGA-FCM with alpha stabilisation,
// epsilon = 0, central differences).
//
// Spline space: degree p, maximum continuity, one open uniform knot vector per direction
// (p + 1 copies of each end of the box, every interior cell face once), so n cells carry
// n + p functions and cell c supports the functions c .. c + p of its direction.
//
// Set-up reuses the set-up of the spectral cell method on the same cells (classification,
// the tree quadrature of every cut cell).  Restricted to one cell, the p + 1 B-splines of a
// direction are polynomials of degree p, so each is the combination of the cell's
// GLL-Lagrange polynomials with coefficients N_{c+j}(x_i) (its values at the cell's GLL
// nodes).  With A_c the tensor product of these 1-D matrices the B-spline element
// matrices are A_c K^L_c A_c^T for the Lagrange ones K^L_c (the uncut reference matrix, or
// the tree-integrated matrix of a cut cell), with the same quadrature; the row sums of the
// B-spline mass are A_c times the row sums of the Lagrange mass (for an uncut cell the GLL
// weights, since GLL quadrature integrates every Lagrange polynomial exactly; for a cut
// cell those of its tree-integrated mass).  Along one direction A_c depends only on the
// cell's position class (p classes at each end, one interior class), so an uncut cell's
// matrix is one of (2p+1)^d class matrices.
//
// Step (eq. cdm in increment form with the row-sum lumped mass): one launch per step.  A
// block owns a tile of DOFs; it stages the u values of the cells that touch the tile (a ring
// of p cells below it) in LDS, forms every such cell's product y_c = K_c u_c (its class
// matrix, or the cut cell's own), and each owned DOF sums the (p+1)^d products of its cells
// in a fixed order (no atomics) before the update of d and u.
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "common.h"
#include "step_common.h"

namespace fcw {

constexpr int kIgaMaxNs = 125;  // (p+1)^d built: 2-D p <= 4, 3-D p <= 3

struct IgaSrc {
  int32_t c[3];
  int32_t pad;
  double f0;
  double b[kIgaMaxNs];  // rho amp N_a(x_s) of the source cell's functions
};

struct IgaCtx {
  int dim = 2, p = 2, precision = FCW_FP64, n_s = 0;
  int n[3] = {1, 1, 1}, nb[3] = {1, 1, 1};
  int64_t ncells = 0, ndof = 0, ncand = 0, n_cut = 0, n_uncut = 0, n_out = 0;
  double lo[3] = {0, 0, 0}, h = 1, rho = 1;
  double dt_crit = 0.0;
  hipStream_t stream = nullptr;
  int64_t footprint = 0;
  int32_t* d_info = nullptr;      // [ncells] -1 out, -2 uncut, >= 0 cut candidate index
  double* d_tab = nullptr;        // [3][2p+1][p+1][p+1] N_{c+j}(x_i), per direction and class
  double* d_kcls64 = nullptr;     // [(2p+1)^d][n_s^2] class matrices
  double* d_rcls = nullptr;       // [(2p+1)^d][n_s] class row sums of the mass
  double* d_kcut64 = nullptr;     // [ncand][n_s^2] cut-cell matrices (zero when all-void)
  double* d_rcut = nullptr;       // [ncand][n_s] cut-cell row sums of the mass
  double* d_mass = nullptr;       // [ndof] row-sum lumped mass
  double* d_sqim = nullptr;       // [ndof] sqrt(1/mass) on active DOFs, 0 elsewhere
  void* d_kcls = nullptr;         // FP32 copies of the matrices (FP32 contexts only)
  void* d_kcut = nullptr;
  void* d_invm = nullptr;
  IgaSrc* d_src = nullptr;        // [kMaxSrc]
  void* d_ubuf = nullptr;         // ping-pong partner of the caller's state
  size_t ubuf_bytes = 0;
  size_t esize() const { return precision == FCW_FP64 ? 8 : 4; }
};

// ---------------------------------------------------------------------------------------
// 1-D B-splines

// Knot m of the open uniform knot vector of n cells of width h from lo (p + 1 end copies).
__device__ static inline double iga_knot(int P, int n, double lo, double h, int m) {
  int k = m - P;
  k = k < 0 ? 0 : (k > n ? n : k);
  return lo + h * k;
}

// Values at x of the P + 1 functions N_c .. N_{c+P} supported on cell c (the pieces of the
// cell's own knot span s = c + P), by the Cox-de Boor recurrence from the degree-0
// indicator of the span: at degree q the functions s - q .. s are nonzero there and
// N_{i,q} = (x - t_i) / (t_{i+q} - t_i) N_{i,q-1} + (t_{i+q+1} - x) / (t_{i+q+1} - t_{i+1}) N_{i+1,q-1}
// with a term of zero width dropped.
__device__ static void iga_cell_basis(int P, int n, double lo, double h, int c, double x,
                                      double* N) {
  double old[kMaxP + 1], cur[kMaxP + 1];
  const int s = c + P;
  old[0] = 1.0;
  for (int q = 1; q <= P; ++q) {
    for (int r = 0; r <= q; ++r) {
      const int i = s - q + r;
      double v = 0.0;
      if (r >= 1) {  // N_{i,q-1} = old[r-1]
        const double ti = iga_knot(P, n, lo, h, i), tq = iga_knot(P, n, lo, h, i + q);
        if (tq > ti) v += (x - ti) / (tq - ti) * old[r - 1];
      }
      if (r <= q - 1) {  // N_{i+1,q-1} = old[r]
        const double t1 = iga_knot(P, n, lo, h, i + 1), tq1 = iga_knot(P, n, lo, h, i + q + 1);
        if (tq1 > t1) v += (tq1 - x) / (tq1 - t1) * old[r];
      }
      cur[r] = v;
    }
    for (int r = 0; r <= q; ++r) old[r] = cur[r];
  }
  for (int j = 0; j <= P; ++j) N[j] = old[j];
}

// Position class of cell c of n along a direction: c (< p) at the low end, p inside,
// 2p - (n - 1 - c) at the high end; a representative cell of each class.
__host__ __device__ static inline int iga_class(int P, int n, int c) {
  return c < P ? c : (c > n - 1 - P ? 2 * P - (n - 1 - c) : P);
}
__host__ __device__ static inline int iga_class_cell(int P, int n, int q) {
  return q < P ? q : (q == P ? P : n - 1 - (2 * P - q));
}

struct TabArgs {
  int dim, P;
  int n[3];
  double lo[3], h;
  const RefTables* ref;
  double* tab;
};

// tab[k][q][j][i] = N_{c+j}(x_i), x_i the GLL nodes of the representative cell c of class q
__global__ void iga_tab_kernel(TabArgs a) {
  const int P = a.P, ncls = 2 * P + 1;
  const int t = threadIdx.x;
  if (t >= a.dim * ncls * (P + 1)) return;
  const int i = t % (P + 1), q = (t / (P + 1)) % ncls, k = t / ((P + 1) * ncls);
  const int c = iga_class_cell(P, a.n[k], q);
  const double x = a.lo[k] + a.h * (c + 0.5 * (a.ref->gll_x[i] + 1.0));
  double N[kMaxP + 1];
  iga_cell_basis(P, a.n[k], a.lo[k], a.h, c, x, N);
  double* out = a.tab + ((size_t)(k * ncls + q) * (P + 1)) * (P + 1);
  for (int j = 0; j <= P; ++j) out[j * (P + 1) + i] = N[j];
}

// ---------------------------------------------------------------------------------------
// Element matrices in the B-spline basis: D = A S A^T and r = A (S_m 1)

struct TransArgs {
  int dim, P, ns;
  int n[3];
  int mode;                 // 0: class matrices (item = class tuple), 1: cut candidates
  int64_t nitems;
  const double* tab;        // [3][2p+1][p+1][p+1]
  const double* src;        // mode 0: K_ref; mode 1: [ncand][n_s^2] Lagrange K_e
  const double* msrc;       // mode 0: GLL lumped diagonal [n_s]; mode 1: [ncand][n_s^2] M_e
  const int32_t* cells;     // mode 1: cell of each candidate
  const int32_t* all_void;  // mode 1: candidate dropped
  double* dst;              // [nitems][n_s^2]
  double* rdst;             // [nitems][n_s]
};

// one workgroup per item; the n_s x n_s matrix in LDS, contracted direction by direction
// (rows and columns of a local index are tensor indices (i0, i1, i2), x fastest)
__global__ __launch_bounds__(256) void iga_transform_kernel(TransArgs a) {
  extern __shared__ double sh[];
  const int ns = a.ns, P = a.P, P1 = P + 1, ncls = 2 * P + 1;
  double* m0 = sh;
  double* m1 = sh + (size_t)ns * ns;
  double* rv = sh + 2 * (size_t)ns * ns;  // [2][ns]
  __shared__ int qk[3];
  const int64_t item = blockIdx.x;
  const int tid = threadIdx.x;
  const double* S;
  bool zero = false;
  if (a.mode == 0) {
    if (tid == 0) {
      int64_t r = item;
      for (int k = 0; k < 3; ++k) { qk[k] = k < a.dim ? (int)(r % ncls) : 0; r /= (k < a.dim ? ncls : 1); }
    }
    S = a.src;
  } else {
    if (tid == 0) {
      int64_t r = a.cells[item];
      for (int k = 0; k < 3; ++k) {
        const int nk = k < a.dim ? a.n[k] : 1;
        const int c = (int)(r % nk);
        r /= nk;
        qk[k] = k < a.dim ? iga_class(P, a.n[k], c) : 0;
      }
    }
    zero = a.all_void[item] != 0;
    S = a.src + (size_t)item * ns * ns;
  }
  __syncthreads();
  double* D = a.dst + (size_t)item * ns * ns;
  double* R = a.rdst + (size_t)item * ns;
  if (zero) {
    for (int e = tid; e < ns * ns; e += blockDim.x) D[e] = 0.0;
    for (int e = tid; e < ns; e += blockDim.x) R[e] = 0.0;
    return;
  }
  for (int e = tid; e < ns * ns; e += blockDim.x) m0[e] = S[e];
  if (a.mode == 0) {
    for (int e = tid; e < ns; e += blockDim.x) rv[e] = a.msrc[e];
  } else {
    const double* M = a.msrc + (size_t)item * ns * ns;
    for (int e = tid; e < ns; e += blockDim.x) {
      double s = 0.0;
      for (int b = 0; b < ns; ++b) s += M[(size_t)e * ns + b];
      rv[e] = s;
    }
  }
  __syncthreads();
  // one 1-D contraction along direction k of the row (side 0) or column (side 1) index:
  // out[.., j_k, ..] = sum_i A_k[j][i] in[.., i, ..]
  double* in = m0;
  double* out = m1;
  int stride = 1;
  for (int k = 0; k < a.dim; ++k) {
    const double* Ak = a.tab + ((size_t)(k * ncls + qk[k]) * P1) * P1;
    for (int side = 0; side < 2; ++side) {
      for (int e = tid; e < ns * ns; e += blockDim.x) {
        const int row = e / ns, col = e % ns;
        const int idx = side == 0 ? row : col;
        const int j = (idx / stride) % P1;
        const int base = idx - j * stride;
        double s = 0.0;
        for (int i = 0; i < P1; ++i) {
          const int src_idx = base + i * stride;
          s += Ak[j * P1 + i] * (side == 0 ? in[src_idx * ns + col] : in[row * ns + src_idx]);
        }
        out[e] = s;
      }
      __syncthreads();
      double* t = in;
      in = out;
      out = t;
    }
    // the row-sum vector takes the row contraction only
    double* rin = rv + (k & 1) * ns;
    double* rout = rv + ((k + 1) & 1) * ns;
    for (int e = tid; e < ns; e += blockDim.x) {
      const int j = (e / stride) % P1;
      const int base = e - j * stride;
      double s = 0.0;
      for (int i = 0; i < P1; ++i) s += Ak[j * P1 + i] * rin[base + i * stride];
      rout[e] = s;
    }
    __syncthreads();
    stride *= P1;
  }
  const double* rfin = rv + (a.dim & 1) * ns;
  for (int e = tid; e < ns * ns; e += blockDim.x) D[e] = in[e];
  for (int e = tid; e < ns; e += blockDim.x) R[e] = rfin[e];
}

// ---------------------------------------------------------------------------------------
// Row-sum lumped mass: per DOF the sum over its kept cells, lower cells first (z, y, x)

struct MassArgsIga {
  int dim, P;
  int n[3], nb[3];
  int64_t ndof;
  const int32_t* info;
  const double* rcls;
  const double* rcut;
  double* mass;
  double* sqim;
};

__global__ void iga_mass_kernel(MassArgsIga a) {
  const int64_t dof = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dof >= a.ndof) return;
  const int P = a.P, P1 = P + 1, ncls = 2 * P + 1;
  const int ns = ipow(P1, a.dim);
  int idx[3] = {0, 0, 0};
  int64_t r = dof;
  for (int k = 0; k < a.dim; ++k) { idx[k] = (int)(r % a.nb[k]); r /= a.nb[k]; }
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < a.dim; ++k) {
    lo[k] = max(idx[k] - P, 0);
    hi[k] = min(idx[k], a.n[k] - 1);
  }
  double m = 0.0;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy)
      for (int cx = lo[0]; cx <= hi[0]; ++cx) {
        const int cc[3] = {cx, cy, cz};
        const int64_t cell = cx + (int64_t)a.n[0] * (cy + (int64_t)a.n[1] * cz);
        const int32_t inf = a.info[cell];
        if (inf == kInfoOut) continue;
        int loc = 0, q = 0, sl = 1, sq = 1;
        for (int k = 0; k < a.dim; ++k) {
          loc += (idx[k] - cc[k]) * sl;
          q += iga_class(P, a.n[k], cc[k]) * sq;
          sl *= P1;
          sq *= ncls;
        }
        m += inf >= 0 ? a.rcut[(size_t)inf * ns + loc] : a.rcls[(size_t)q * ns + loc];
      }
  a.mass[dof] = m;
  a.sqim[dof] = m > 0.0 ? sqrt(1.0 / m) : 0.0;
}

template <typename T>
__global__ void iga_invm_kernel(const double* mass, T* invm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) invm[i] = mass[i] > 0.0 ? (T)(1.0 / mass[i]) : (T)0;
}

template <typename T>
__global__ void iga_cast_kernel(const double* s, T* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (T)s[i];
}

// ---------------------------------------------------------------------------------------
// Point sources: the source cell (lo_k <= x_k < lo_k + h, clamped to the grid) and
// b_a = rho amp N_a(x_s)

struct SrcArgsIga {
  int dim, P, nsrc;
  int n[3];
  double lo[3], h, rho;
  double x[kMaxSrc][3];
  double amp[kMaxSrc], f0[kMaxSrc];
  IgaSrc* out;
};

__global__ void iga_source_kernel(SrcArgsIga a) {
  const int s = blockIdx.x;
  if (s >= a.nsrc || threadIdx.x != 0) return;
  const int P = a.P, P1 = P + 1;
  double N[3][kMaxP + 1];
  IgaSrc& o = a.out[s];
  for (int k = 0; k < 3; ++k) {
    if (k < a.dim) {
      int c = (int)floor((a.x[s][k] - a.lo[k]) / a.h);
      c = c < 0 ? 0 : (c > a.n[k] - 1 ? a.n[k] - 1 : c);
      o.c[k] = c;
      iga_cell_basis(P, a.n[k], a.lo[k], a.h, c, a.x[s][k], N[k]);
    } else {
      o.c[k] = 0;
      N[k][0] = 1.0;
    }
  }
  o.f0 = a.f0[s];
  const int ns = ipow(P1, a.dim);
  for (int e = 0; e < ns; ++e) {
    const int j0 = e % P1, j1 = (e / P1) % P1, j2 = e / (P1 * P1);
    o.b[e] = a.rho * a.amp[s] * (N[0][j0] * (a.dim > 1 ? N[1][j1] : 1.0)) *
             (a.dim > 2 ? N[2][j2] : 1.0);
  }
}

// ---------------------------------------------------------------------------------------
// The step kernel

template <typename T>
struct IgaStepArgs {
  int n[3], nb[3];
  int64_t ndof;
  const int32_t* info;
  const T* kcls;   // [(2p+1)^d][n_s^2]
  const T* kint;   // the interior class matrix
  const T* kcut;   // [ncand][n_s^2]
  const T* invm;   // [ndof]
  const T* uin;    // [nrhs][ndof]
  T* uout;         // [nrhs][ndof] (apply: K u)
  T* d;            // [nrhs][ndof]
  const IgaSrc* src;
  double t, dt2;   // source time; the factor of the acceleration (dt^2, dt^2/2 at start)
  int apply;       // 1: uout = K uin only
};

template <typename T, int DIM, int P>
struct IgaTile;
template <typename T, int P>
struct IgaTile<T, 2, P> { static constexpr int TX = 16, TY = 16, TZ = 1; };
template <typename T>
struct IgaTile<T, 3, 2> { static constexpr int TX = 6, TY = 6, TZ = 6; };
template <>
struct IgaTile<float, 3, 3> { static constexpr int TX = 4, TY = 4, TZ = 4; };
template <>
struct IgaTile<double, 3, 3> { static constexpr int TX = 4, TY = 4, TZ = 2; };

template <typename T, int DIM, int P>
struct IgaShape {
  static constexpr int P1 = P + 1;
  static constexpr int NS = DIM == 2 ? P1 * P1 : P1 * P1 * P1;
  static constexpr int TX = IgaTile<T, DIM, P>::TX, TY = IgaTile<T, DIM, P>::TY,
                       TZ = IgaTile<T, DIM, P>::TZ;
  static constexpr int CX = TX + P, CY = TY + P, CZ = DIM == 3 ? TZ + P : 1;  // cells
  static constexpr int UX = TX + 2 * P, UY = TY + 2 * P, UZ = DIM == 3 ? TZ + 2 * P : 1;
  static constexpr int NCR = CX * CY * CZ, NUR = UX * UY * UZ, NOWN = TX * TY * TZ;
  static constexpr int NCLS = 2 * P + 1;
  static constexpr int QINT = DIM == 2 ? P + NCLS * P : P + NCLS * (P + NCLS * P);
  // matrix-core form of the interior class: 16-cell batches, K in NMB x NKS A fragments
  static constexpr int NMB = (NS + 15) / 16, NKS = (NS + 3) / 4;
  static constexpr bool MF = NMB * NKS <= 32;
  static constexpr int NSP = NS | 1;  // product stride per cell (odd: conflict-free)
  static constexpr size_t lds_bytes() {
    return ((size_t)NUR + (size_t)NCR * NSP) * sizeof(T) + (size_t)(2 * NCR + 1) * 4;
  }
};

template <typename T, int DIM, int P>
__global__ __launch_bounds__(256) void iga_step_kernel(IgaStepArgs<T> a) {
  using S = IgaShape<T, DIM, P>;
  constexpr int P1 = S::P1, NS = S::NS;
  extern __shared__ __attribute__((aligned(16))) unsigned char iga_lds[];
  T* us = reinterpret_cast<T*>(iga_lds);  // [UZ][UY][UX]
  T* ys = us + S::NUR;                    // [NCR][NSP]
  int* cin = reinterpret_cast<int*>(ys + (size_t)S::NCR * S::NSP);  // [NCR] cell codes
  int* glist = cin + S::NCR;  // [NCR] cells with their own matrix (cut, boundary class)
  int* gcnt = glist + S::NCR;
  constexpr int NSP = S::NSP;
  static_assert(NS <= 64, "one row per lane in the per-cell matrix products");
  const int tid = threadIdx.x;
  const int rhs = DIM == 3 ? (int)blockIdx.z / ((a.nb[2] + S::TZ - 1) / S::TZ) : (int)blockIdx.z;
  const int bz = DIM == 3 ? (int)blockIdx.z % ((a.nb[2] + S::TZ - 1) / S::TZ) : 0;
  const int X0 = blockIdx.x * S::TX, Y0 = blockIdx.y * S::TY, Z0 = bz * S::TZ;
  const int64_t off = (int64_t)rhs * a.ndof;
  const T* u = a.uin + off;
  // the owned DOF's update operands go first (in flight through the product phases)
  const int ox = tid % S::TX, oy = (tid / S::TX) % S::TY, oz = tid / (S::TX * S::TY);
  const int gx = X0 + ox, gy = Y0 + oy, gz = Z0 + oz;
  const bool own = tid < S::NOWN && gx < a.nb[0] && gy < a.nb[1] && gz < a.nb[2];
  const int64_t g = own ? gx + (int64_t)a.nb[0] * (gy + (int64_t)a.nb[1] * gz) : 0;
  T d_own = (T)0, im_own = (T)0;
  if (own && !a.apply) {
    d_own = a.d[off + g];
    im_own = a.invm[g];
  }
  // the interior matrix as MFMA A fragments (lane lc + 16 lk holds K_int[16 mb + lc][4 kk +
  // lk]) and the LDS offsets of this lane's B rows (function 4 kk + lk of a cell)
  constexpr int NMBX = S::MF ? S::NMB : 1, NKSX = S::MF ? S::NKS : 1;
  T areg[NMBX][NKSX];
  int offk[NKSX];
  if constexpr (S::MF) {
    const int lc = tid & 15, lk = (tid & 63) >> 4;
#pragma unroll
    for (int kk = 0; kk < S::NKS; ++kk) {
      const int e = 4 * kk + lk;
      const int ee = e < NS ? e : 0;  // padded k rows read a real value (A is zero there)
      const int jx = ee % P1, jy = (ee / P1) % P1, jz = ee / (P1 * P1);
      offk[kk] = jx + S::UX * (jy + S::UY * (DIM == 3 ? jz : 0));
#pragma unroll
      for (int mb = 0; mb < S::NMB; ++mb) {
        const int r = mb * 16 + lc;
        areg[mb][kk] = (r < NS && e < NS) ? a.kint[r * NS + e] : (T)0;
      }
    }
  }
  // u of the DOFs [X0 - P, X0 + TX + P) (per direction), zero outside the grid
  for (int e = tid; e < S::NUR; e += 256) {
    const int ex = e % S::UX, ey = (e / S::UX) % S::UY, ez = e / (S::UX * S::UY);
    const int hx = X0 - P + ex, hy = Y0 - P + ey, hz = Z0 - (DIM == 3 ? P : 0) + ez;
    const bool in = hx >= 0 && hx < a.nb[0] && hy >= 0 && hy < a.nb[1] && hz >= 0 &&
                    hz < a.nb[2];
    us[e] = in ? u[hx + (int64_t)a.nb[0] * (hy + (int64_t)a.nb[1] * hz)] : (T)0;
  }
  // codes of the cells [X0 - P, X0 + TX) (per direction): kInfoOut, kInfoUncut for the
  // interior class, the cut candidate (>= 0), or -3 - q for an uncut cell of class q
  for (int cl = tid; cl < S::NCR; cl += 256) {
    const int lx = cl % S::CX, ly = (cl / S::CX) % S::CY, lz = cl / (S::CX * S::CY);
    const int cx = X0 - P + lx, cy = Y0 - P + ly, cz = Z0 - (DIM == 3 ? P : 0) + lz;
    int32_t inf = kInfoOut;
    if (cx >= 0 && cx < a.n[0] && cy >= 0 && cy < a.n[1] && cz >= 0 && cz < a.n[2])
      inf = a.info[cx + (int64_t)a.n[0] * (cy + (int64_t)a.n[1] * cz)];
    if (inf == kInfoUncut) {
      int q = iga_class(P, a.n[0], cx) + S::NCLS * iga_class(P, a.n[1], cy);
      if (DIM == 3) q += S::NCLS * S::NCLS * iga_class(P, a.n[2], cz);
      if (q != S::QINT) inf = -3 - q;
    }
    cin[cl] = inf;
  }
  __syncthreads();
  if (tid < 64) {
    // wave 0 lists the cells with their own matrix, in region order
    int base = 0;
    for (int c0 = 0; c0 < S::NCR; c0 += 64) {
      const int cl = c0 + tid;
      const int v = cl < S::NCR ? cin[cl] : kInfoOut;
      const bool g = v >= 0 || v <= -3;
      const unsigned long long m = __ballot(g);
      if (g) glist[base + __popcll(m & ((1ull << tid) - 1ull))] = cl;
      base += __popcll(m);
    }
    if (tid == 0) *gcnt = base;
  }
  if constexpr (S::MF) {
    // interior-class cells on the matrix cores: Y (NS x 16 cells) = K_int U, lane lc + 16 lk
    // holds K_int[16 mb + lc][4 kk + lk] and u of cell 16 b + lc at function 4 kk + lk
    const int lane = tid & 63, wave = tid >> 6, lc = lane & 15, lk = lane >> 4;
    constexpr int NB = (S::NCR + 15) / 16;
    for (int b = wave; b < NB; b += 4) {
      const int cl = min(b * 16 + lc, S::NCR - 1);
      const int lx = cl % S::CX, ly = (cl / S::CX) % S::CY, lz = cl / (S::CX * S::CY);
      const int base = lx + S::UX * (ly + S::UY * lz);
      T bv[S::NKS];
#pragma unroll
      for (int kk = 0; kk < S::NKS; ++kk) bv[kk] = us[base + offk[kk]];
      const bool mine = b * 16 + lc < S::NCR && cin[cl] == kInfoUncut;
#pragma unroll
      for (int mb = 0; mb < S::NMB; ++mb) {
        typename Mma<T>::acc acc = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < S::NKS; ++kk) acc = Mma<T>::mma(areg[mb][kk], bv[kk], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mb * 16 + Mma<T>::row(lk, r);
          if (mine && row < NS) ys[(size_t)cl * NSP + row] = acc[r];
        }
      }
    }
  }
  // outside cells: zeros; without the matrix-core form, interior cells one per thread
  for (int cl = tid; cl < S::NCR; cl += 256) {
    const int inf = cin[cl];
    T* y = ys + (size_t)cl * NSP;
    if (inf == kInfoOut) {
      for (int i = 0; i < NS; ++i) y[i] = (T)0;
    } else if (!S::MF && inf == kInfoUncut) {
      const int lx = cl % S::CX, ly = (cl / S::CX) % S::CY, lz = cl / (S::CX * S::CY);
      T ue[NS];
#pragma unroll
      for (int e = 0; e < NS; ++e) {
        const int jx = e % P1, jy = (e / P1) % P1, jz = e / (P1 * P1);
        ue[e] = us[(lx + jx) + S::UX * ((ly + jy) + S::UY * (lz + (DIM == 3 ? jz : 0)))];
      }
      // one matrix for every lane on this path (uniform loads)
      for (int i = 0; i < NS; ++i) {
        T acc = (T)0;
#pragma unroll
        for (int j = 0; j < NS; ++j) acc += a.kint[i * NS + j] * ue[j];
        y[i] = acc;
      }
    }
  }
  __syncthreads();
  // cells with their own matrix (cut cells; uncut cells of a boundary class): LPC lanes
  // per cell, lane r forms row r with all NS matrix loads issued together
  {
    constexpr int LPC = NS <= 32 ? 32 : 64;
    const int lane = tid & 63, wave = tid >> 6;
    const int r = lane % LPC, slot = lane / LPC;
    const int ng = *gcnt;
    for (int g0 = (wave * 64 / LPC); g0 < ng; g0 += 4 * 64 / LPC) {
      const int gi = g0 + slot;
      if (gi >= ng || r >= NS) continue;
      const int cl = glist[gi];
      const int inf = cin[cl];
      const T* K = inf >= 0 ? a.kcut + (size_t)inf * NS * NS
                            : a.kcls + (size_t)(-3 - inf) * NS * NS;
      T kr[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) kr[j] = K[(size_t)r * NS + j];
      const int lx = cl % S::CX, ly = (cl / S::CX) % S::CY, lz = cl / (S::CX * S::CY);
      T acc = (T)0;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int jx = j % P1, jy = (j / P1) % P1, jz = j / (P1 * P1);
        acc += kr[j] * us[(lx + jx) + S::UX * ((ly + jy) + S::UY * (lz + (DIM == 3 ? jz : 0)))];
      }
      ys[(size_t)cl * NSP + r] = acc;
    }
  }
  __syncthreads();
  if (!own) return;
  // the cells of this DOF: local cell ox + P - jx for jx = 0..P (lower cells first)
  T acc = (T)0;
  for (int jz = (DIM == 3 ? P : 0); jz >= 0; --jz)
    for (int jy = P; jy >= 0; --jy)
#pragma unroll
      for (int jx = P; jx >= 0; --jx) {
        const int cl = (ox + P - jx) + S::CX * ((oy + P - jy) + S::CY * (oz + (DIM == 3 ? P : 0) - jz));
        acc += ys[(size_t)cl * NSP + jx + P1 * (jy + P1 * jz)];
      }
  if (a.apply) {
    a.uout[off + g] = acc;
    return;
  }
  T F = (T)0;
  const IgaSrc& s = a.src[rhs];
  const int sx = gx - s.c[0], sy = gy - s.c[1], sz = gz - s.c[2];
  if (sx >= 0 && sx <= P && sy >= 0 && sy <= P && (DIM == 2 || (sz >= 0 && sz <= P)))
    F = (T)(ricker(a.t, s.f0) * s.b[sx + P1 * (sy + P1 * (DIM == 3 ? sz : 0))]);
  const T dn = d_own + (T)a.dt2 * im_own * (F - acc);
  a.d[off + g] = dn;
  a.uout[off + g] = us[(ox + P) + S::UX * ((oy + P) + S::UY * (oz + (DIM == 3 ? P : 0)))] + dn;
}

// ---------------------------------------------------------------------------------------
// launchers

template <typename T, int DIM, int P>
static fcw_status iga_launch_t(IgaCtx& c, int nrhs, const void* uin, void* uout, void* d,
                               double t, double dt2, int apply) {
  using S = IgaShape<T, DIM, P>;
  static_assert(S::lds_bytes() <= 160 * 1024, "LDS");
  static bool attr = false;
  if (!attr) {
    FCW_HIP(hipFuncSetAttribute((const void*)iga_step_kernel<T, DIM, P>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::lds_bytes()));
    attr = true;
  }
  IgaStepArgs<T> a{};
  for (int k = 0; k < 3; ++k) { a.n[k] = c.n[k]; a.nb[k] = c.nb[k]; }
  a.ndof = c.ndof;
  a.info = c.d_info;
  // the FP64 kernel (FP64 steps, and the Lanczos operator of every context) reads the FP64
  // matrices; the step-precision copies serve FP32 steps; the inverse mass is read by steps
  // only, which run in the context's precision
  const bool f64 = std::is_same<T, double>::value;
  a.kcls = f64 ? (const T*)c.d_kcls64 : (const T*)c.d_kcls;
  a.kint = a.kcls + (size_t)S::QINT * S::NS * S::NS;
  a.kcut = f64 ? (const T*)c.d_kcut64 : (const T*)c.d_kcut;
  a.invm = (const T*)c.d_invm;
  if (!apply && (int)c.esize() != (int)sizeof(T)) {
    set_error("IGA step kernel precision differs from the context's");
    return FCW_E_STATE;
  }
  a.uin = (const T*)uin;
  a.uout = (T*)uout;
  a.d = (T*)d;
  a.src = c.d_src;
  a.t = t;
  a.dt2 = dt2;
  a.apply = apply;
  const int gz = DIM == 3 ? (c.nb[2] + S::TZ - 1) / S::TZ : 1;
  dim3 grid((c.nb[0] + S::TX - 1) / S::TX, (c.nb[1] + S::TY - 1) / S::TY, gz * nrhs);
  iga_step_kernel<T, DIM, P><<<grid, 256, S::lds_bytes(), c.stream>>>(a);
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

template <typename T>
static fcw_status iga_launch_p(IgaCtx& c, int nrhs, const void* uin, void* uout, void* d,
                               double t, double dt2, int apply) {
  if (c.dim == 2) {
    switch (c.p) {
      case 2: return iga_launch_t<T, 2, 2>(c, nrhs, uin, uout, d, t, dt2, apply);
      case 3: return iga_launch_t<T, 2, 3>(c, nrhs, uin, uout, d, t, dt2, apply);
      case 4: return iga_launch_t<T, 2, 4>(c, nrhs, uin, uout, d, t, dt2, apply);
    }
  } else {
    switch (c.p) {
      case 2: return iga_launch_t<T, 3, 2>(c, nrhs, uin, uout, d, t, dt2, apply);
      case 3: return iga_launch_t<T, 3, 3>(c, nrhs, uin, uout, d, t, dt2, apply);
    }
  }
  set_error("no IGA step kernel for dim=%d p=%d", c.dim, c.p);
  return FCW_E_UNSUPPORTED;
}

static fcw_status iga_launch(IgaCtx& c, int nrhs, const void* uin, void* uout, void* d, double t,
                             double dt2, int apply) {
  return c.precision == FCW_FP64 ? iga_launch_p<double>(c, nrhs, uin, uout, d, t, dt2, apply)
                                 : iga_launch_p<float>(c, nrhs, uin, uout, d, t, dt2, apply);
}

static bool iga_supported(int dim, int p) {
  return (dim == 2 && p >= 2 && p <= 4) || (dim == 3 && p >= 2 && p <= 3);
}

// FP64 operator of the Lanczos iteration: w = S K S v, S = diag(sqrt(1/m))
__global__ void iga_scale_kernel(const double* s, const double* v, double* w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = s[i] * v[i];
}

struct IgaLanczosArg {
  IgaCtx* c;
  double* tmp;
  double* kv;
};

static fcw_status iga_apply_scaled(void* arg, const double* v, double* w) {
  IgaLanczosArg& a = *(IgaLanczosArg*)arg;
  IgaCtx& c = *a.c;
  const unsigned g = (unsigned)((c.ndof + 255) / 256);
  iga_scale_kernel<<<g, 256, 0, c.stream>>>(c.d_sqim, v, a.tmp, c.ndof);
  FCW_HIP(hipGetLastError());
  fcw_status st = iga_launch_p<double>(c, 1, a.tmp, a.kv, nullptr, 0.0, 0.0, 1);
  if (st) return st;
  iga_scale_kernel<<<g, 256, 0, c.stream>>>(c.d_sqim, a.kv, w, c.ndof);
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

template <typename P>
static fcw_status iga_malloc(IgaCtx& c, P** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  c.footprint += (int64_t)bytes;
  return FCW_OK;
}

static void iga_free(IgaCtx& c) {
  void* ps[] = {c.d_info, c.d_tab, c.d_kcls64, c.d_rcls, c.d_kcut64, c.d_rcut, c.d_mass,
                c.d_sqim, c.d_kcls, c.d_kcut, c.d_invm, c.d_src, c.d_ubuf};
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

}  // namespace fcw

struct fcw_iga : public fcw::IgaCtx {};

using namespace fcw;

extern "C" {

fcw_status fcw_iga_create(fcw_ctx* cells, fcw_iga** out) {
  clear_error();
  if (!cells || !out) { set_error("null argument"); return FCW_E_ARG; }
  *out = nullptr;
  Ctx& s = *cells;
  if (s.poisoned) { set_error("context poisoned by an earlier device error"); return FCW_E_DEVICE; }
  if (s.state < 1) { set_error("cells not assembled"); return FCW_E_STATE; }
  if (s.ncomp != 1) { set_error("IGA-FCM is built for the scalar wave equation"); return FCW_E_UNSUPPORTED; }
  if (!iga_supported(s.dim, s.p)) {
    set_error("no IGA step kernel for dim=%d p=%d (2-D p 2..4, 3-D p 2..3)", s.dim, s.p);
    return FCW_E_UNSUPPORTED;
  }
  if (s.precision != FCW_FP64 && s.precision != FCW_FP32) {
    set_error("IGA-FCM steps in FP64 or FP32");
    return FCW_E_UNSUPPORTED;
  }
  for (int k = 0; k < s.dim; ++k)
    if (s.ncells[k] < 2 * s.p + 1) {
      set_error("IGA-FCM needs at least 2p+1 cells per direction (got %d)", s.ncells[k]);
      return FCW_E_ARG;
    }
  fcw_iga* g = new (std::nothrow) fcw_iga();
  if (!g) { set_error("host allocation failed"); return FCW_E_NOMEM; }
  IgaCtx& c = *g;
  c.dim = s.dim;
  c.p = s.p;
  c.precision = s.precision;
  c.n_s = s.n_s;
  c.ndof = 1;
  for (int k = 0; k < 3; ++k) {
    c.n[k] = s.ncells[k];
    c.nb[k] = k < s.dim ? s.ncells[k] + s.p : 1;
    c.lo[k] = s.lo[k];
    c.ndof *= c.nb[k];
  }
  c.ncells = s.ncell_total;
  c.ncand = s.n_cut_cand;
  c.n_cut = s.n_cut;
  c.n_uncut = s.n_uncut;
  c.n_out = s.n_out;
  c.h = s.h;
  c.rho = s.rho;
  c.stream = s.stream;
  auto fail = [&](fcw_status st) {
    iga_free(c);
    delete g;
    return st;
  };
  const int ncls = 2 * c.p + 1;
  const int64_t nq = ipow(ncls, c.dim);
  const size_t ns = c.n_s, ns2 = ns * ns, es = c.esize();
  const size_t nc = (size_t)(c.ncand > 0 ? c.ncand : 1);
  fcw_status st;
  if ((st = iga_malloc(c, &c.d_info, (size_t)c.ncells * 4)) ||
      (st = iga_malloc(c, &c.d_tab, (size_t)3 * ncls * (c.p + 1) * (c.p + 1) * 8)) ||
      (st = iga_malloc(c, &c.d_kcls64, nq * ns2 * 8)) || (st = iga_malloc(c, &c.d_rcls, nq * ns * 8)) ||
      (st = iga_malloc(c, &c.d_kcut64, nc * ns2 * 8)) || (st = iga_malloc(c, &c.d_rcut, nc * ns * 8)) ||
      (st = iga_malloc(c, &c.d_mass, (size_t)c.ndof * 8)) ||
      (st = iga_malloc(c, &c.d_sqim, (size_t)c.ndof * 8)) ||
      (c.precision != FCW_FP64 && ((st = iga_malloc(c, &c.d_kcls, nq * ns2 * es)) ||
                                    (st = iga_malloc(c, &c.d_kcut, nc * ns2 * es)))) ||
      (st = iga_malloc(c, &c.d_invm, (size_t)c.ndof * es)) ||
      (st = iga_malloc(c, &c.d_src, (size_t)kMaxSrc * sizeof(IgaSrc))))
    return fail(st);
  auto hip = [&](hipError_t e, const char* what) { return e == hipSuccess ? FCW_OK : hip_fail(e, what); };
  if ((st = hip(hipMemcpyAsync(c.d_info, s.d_info, (size_t)c.ncells * 4, hipMemcpyDeviceToDevice,
                               c.stream), "hipMemcpyAsync")))
    return fail(st);
  TabArgs ta{};
  ta.dim = c.dim;
  ta.P = c.p;
  for (int k = 0; k < 3; ++k) { ta.n[k] = c.n[k]; ta.lo[k] = c.lo[k]; }
  ta.h = c.h;
  ta.ref = s.d_tab;
  ta.tab = c.d_tab;
  iga_tab_kernel<<<1, 256, 0, c.stream>>>(ta);
  if ((st = hip(hipGetLastError(), "iga_tab_kernel"))) return fail(st);
  const size_t lds = (2 * ns2 + 2 * ns) * 8;
  if ((st = hip(hipFuncSetAttribute((const void*)iga_transform_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                "hipFuncSetAttribute")))
    return fail(st);
  TransArgs tr{};
  tr.dim = c.dim;
  tr.P = c.p;
  tr.ns = c.n_s;
  for (int k = 0; k < 3; ++k) tr.n[k] = c.n[k];
  tr.tab = c.d_tab;
  tr.mode = 0;
  tr.nitems = nq;
  tr.src = s.d_kref;
  tr.msrc = s.d_lref;
  tr.dst = c.d_kcls64;
  tr.rdst = c.d_rcls;
  iga_transform_kernel<<<(unsigned)nq, 256, lds, c.stream>>>(tr);
  if ((st = hip(hipGetLastError(), "iga_transform_kernel"))) return fail(st);
  if (c.ncand > 0) {
    tr.mode = 1;
    tr.nitems = c.ncand;
    tr.src = s.d_kcut;
    tr.msrc = s.d_mcut;
    tr.cells = s.d_cut_cells;
    tr.all_void = s.d_all_void;
    tr.dst = c.d_kcut64;
    tr.rdst = c.d_rcut;
    iga_transform_kernel<<<(unsigned)c.ncand, 256, lds, c.stream>>>(tr);
    if ((st = hip(hipGetLastError(), "iga_transform_kernel"))) return fail(st);
  }
  MassArgsIga ma{};
  ma.dim = c.dim;
  ma.P = c.p;
  for (int k = 0; k < 3; ++k) { ma.n[k] = c.n[k]; ma.nb[k] = c.nb[k]; }
  ma.ndof = c.ndof;
  ma.info = c.d_info;
  ma.rcls = c.d_rcls;
  ma.rcut = c.d_rcut;
  ma.mass = c.d_mass;
  ma.sqim = c.d_sqim;
  const unsigned gd = (unsigned)((c.ndof + 255) / 256);
  iga_mass_kernel<<<gd, 256, 0, c.stream>>>(ma);
  if ((st = hip(hipGetLastError(), "iga_mass_kernel"))) return fail(st);
  const int64_t nkc = nq * (int64_t)ns2, nkk = (int64_t)nc * ns2;
  if (c.precision == FCW_FP64) {
    iga_invm_kernel<double><<<gd, 256, 0, c.stream>>>(c.d_mass, (double*)c.d_invm, c.ndof);
  } else {
    iga_invm_kernel<float><<<gd, 256, 0, c.stream>>>(c.d_mass, (float*)c.d_invm, c.ndof);
    iga_cast_kernel<float><<<(unsigned)((nkc + 255) / 256), 256, 0, c.stream>>>(c.d_kcls64, (float*)c.d_kcls, nkc);
    iga_cast_kernel<float><<<(unsigned)((nkk + 255) / 256), 256, 0, c.stream>>>(c.d_kcut64, (float*)c.d_kcut, nkk);
  }
  if ((st = hip(hipGetLastError(), "iga_cast_kernel"))) return fail(st);
  if ((st = hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize"))) return fail(st);
  *out = g;
  return FCW_OK;
}

void fcw_iga_destroy(fcw_iga* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  iga_free(*g);
  delete g;
}

fcw_status fcw_iga_query(const fcw_iga* g, fcw_iga_info* info) {
  clear_error();
  if (!g || !info) { set_error("null argument"); return FCW_E_ARG; }
  info->ndof = g->ndof;
  for (int k = 0; k < 3; ++k) info->nbasis[k] = g->nb[k];
  info->n_s = g->n_s;
  info->precision = g->precision;
  info->n_cut = g->n_cut;
  info->n_uncut = g->n_uncut;
  info->n_out = g->n_out;
  info->dt_crit = g->dt_crit;
  info->footprint_bytes = g->footprint;
  return FCW_OK;
}

fcw_status fcw_iga_critical_dt(fcw_iga* g, int32_t max_iter, double rtol, double* dt_crit) {
  clear_error();
  if (!g || !dt_crit || max_iter < 2 || !(rtol > 0.0)) { set_error("invalid argument"); return FCW_E_ARG; }
  IgaCtx& c = *g;
  IgaLanczosArg arg{&c, nullptr, nullptr};
  FCW_HIP(hipMallocAsync((void**)&arg.tmp, (size_t)c.ndof * 8, c.stream));
  FCW_HIP(hipMallocAsync((void**)&arg.kv, (size_t)c.ndof * 8, c.stream));
  LanczosOp op{c.stream, c.ndof, c.d_sqim, c.ndof, 1, iga_apply_scaled, &arg};
  double lmax = 0.0;
  fcw_status st = lanczos_run(op, max_iter, rtol, &lmax);
  (void)hipFreeAsync(arg.tmp, c.stream);
  (void)hipFreeAsync(arg.kv, c.stream);
  FCW_HIP(hipStreamSynchronize(c.stream));
  if (st) return st;
  c.dt_crit = 2.0 / sqrt(lmax);
  *dt_crit = c.dt_crit;
  return FCW_OK;
}

fcw_status fcw_iga_apply_stiffness(fcw_iga* g, int32_t nrhs, const void* u, void* r) {
  clear_error();
  if (!g || !u || !r || nrhs < 1 || nrhs > kMaxSrc) { set_error("invalid argument"); return FCW_E_ARG; }
  return iga_launch(*g, nrhs, u, r, nullptr, 0.0, 0.0, 1);
}

fcw_status fcw_iga_step(fcw_iga* g, int32_t nrhs, void* u, void* d, const fcw_source* src,
                        double t0, double dt, int32_t nsteps, int32_t start) {
  clear_error();
  if (!g || !u || !d || !src || nrhs < 1 || nrhs > kMaxSrc || nsteps < 0 || !(dt > 0.0)) {
    set_error("invalid argument");
    return FCW_E_ARG;
  }
  IgaCtx& c = *g;
  SrcArgsIga sa{};
  sa.dim = c.dim;
  sa.P = c.p;
  sa.nsrc = nrhs;
  for (int k = 0; k < 3; ++k) { sa.n[k] = c.n[k]; sa.lo[k] = c.lo[k]; }
  sa.h = c.h;
  sa.rho = c.rho;
  for (int r = 0; r < nrhs; ++r) {
    if (src[r].sigma > 0.0) { set_error("volumetric sources are not built for IGA-FCM"); return FCW_E_UNSUPPORTED; }
    for (int k = 0; k < 3; ++k) {
      sa.x[r][k] = k < c.dim ? src[r].x[k] : 0.0;
      if (k < c.dim && !(src[r].x[k] >= c.lo[k] && src[r].x[k] <= c.lo[k] + c.n[k] * c.h)) {
        set_error("source %d outside the box", r);
        return FCW_E_ARG;
      }
    }
    sa.amp[r] = src[r].amp;
    sa.f0[r] = src[r].f0;
  }
  sa.out = c.d_src;
  iga_source_kernel<<<nrhs, 64, 0, c.stream>>>(sa);
  FCW_HIP(hipGetLastError());
  if (nsteps == 0) return FCW_OK;
  const size_t bytes = (size_t)nrhs * c.ndof * c.esize();
  if (bytes > c.ubuf_bytes) {
    if (c.d_ubuf) FCW_HIP(hipFree(c.d_ubuf));
    c.d_ubuf = nullptr;
    c.ubuf_bytes = 0;
    FCW_HIP(hipMalloc(&c.d_ubuf, bytes));
    c.ubuf_bytes = bytes;
  }
  void* cur = u;
  void* nxt = c.d_ubuf;
  for (int k = 0; k < nsteps; ++k) {
    const double f = (start && k == 0) ? 0.5 : 1.0;
    fcw_status st = iga_launch(c, nrhs, cur, nxt, d, t0 + k * dt, f * dt * dt, 0);
    if (st) return st;
    void* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (cur != u) FCW_HIP(hipMemcpyAsync(u, cur, bytes, hipMemcpyDeviceToDevice, c.stream));
  return FCW_OK;
}

fcw_status fcw_iga_export(const fcw_iga* g, int32_t which, void* dst, int64_t capacity,
                          int64_t* count) {
  clear_error();
  if (!g) { set_error("null argument"); return FCW_E_ARG; }
  const IgaCtx& c = *g;
  const void* srcp = nullptr;
  int64_t n = 0;
  const int64_t ns2 = (int64_t)c.n_s * c.n_s;
  switch (which) {
    case FCW_IGA_ARR_MASS: srcp = c.d_mass; n = c.ndof; break;
    case FCW_IGA_ARR_K_CLASS: srcp = c.d_kcls64; n = ipow(2 * c.p + 1, c.dim) * ns2; break;
    case FCW_IGA_ARR_K_CUT: srcp = c.d_kcut64; n = c.ncand * ns2; break;
    default: set_error("unknown array %d", which); return FCW_E_ARG;
  }
  if (count) *count = n;
  if (!dst) return FCW_OK;
  if (capacity < n) {
    set_error("capacity %lld < %lld", (long long)capacity, (long long)n);
    return FCW_E_ARG;
  }
  if (n == 0) return FCW_OK;
  FCW_HIP(hipMemcpyAsync(dst, srcp, (size_t)n * 8, hipMemcpyDeviceToHost, c.stream));
  FCW_HIP(hipStreamSynchronize(c.stream));
  return FCW_OK;
}

}  // extern "C"
