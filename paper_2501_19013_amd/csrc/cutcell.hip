// Cut-cell products y_e = K_e u_e of one step (paper eq. semi, the cut-cell part of
// K u), computed once per cut cell ahead of the tile kernels.
//
// The tile kernels give every owned node all of its cells by staging one ring of cells
// around the tile, so cells on a tile's low faces are visited by two (2-D) to eight
// (3-D) tiles.  For uncut cells that repeat costs matrix-core time only; for cut cells
// it would repeat the stream of their own matrices, the dominant HBM traffic of 3-D
// problems, and it would put long dependent FP64 loops into the tile kernels.  This
// kernel streams each packed K_e exactly once per step:
//
//  * one wave per cut cell; the packed upper triangle (column-major) goes global ->
//    LDS with global_load_lds (64 coalesced dwords per instruction, no registers);
//  * the cell's node values are gathered once per right-hand side and broadcast from
//    LDS; lane i accumulates row i of K_e u_e in FP64 over the columns in order;
//  * y_e (state precision) is written to [nrhs][n_cut_cand][n_loc], where the tile
//    kernels add it to their node sums in their fixed order.
//
// Several problems of one kind share a launch through an array of problem records
// (blocks are assigned to problems by prefix offsets), like the batched tile kernels.
#include <algorithm>
#include <cstring>

#include "step_common.h"

namespace fcw {

template <typename T>
struct CutProb {
  const T* ua;               // ping-pong pair of the state: step j of a call reads
  const T* ub;               // ((nsteps - 1 - j) & 1) ? ua : ub
  const T* kcut;             // [ncand][npk] packed upper, column-major
  const int32_t* cut_cells;  // [ncand]
  const int32_t* info;       // [ncells]
  T* y;                      // [nrhs][ncand][n_loc]
  int64_t ncand, nnodes, ndof;
  int64_t blk0;              // first block of this problem in a batched launch
  int n[3], np[3];
  int nrhs, nsteps;
};

template <typename T, int NL>
struct CutShape {
  static constexpr int DPE = (int)(sizeof(T) / 4);
  static constexpr int KD = NL * (NL + 1) / 2 * DPE;  // dwords per packed matrix
  static constexpr int KDP = (KD + 63) / 64 * 64;
  static constexpr int UEP = (NL * DPE + 63) / 64 * 64;
  // Pipelined form, for matrices of 1024 to 4096 dwords: a wave walks CPW cells; the
  // next cell's packed matrix travels global -> registers while the current one is
  // reduced from LDS (node values kept there in FP64).  Other sizes: packed triangle
  // global -> LDS directly, one cell per wave.
  static constexpr bool PIPE = KDP / 64 <= 64 && KD >= 1024;
  static constexpr int STRIDE = KDP + (PIPE ? (2 * NL + 63) / 64 * 64 : UEP);  // LDS dwords per wave
  static constexpr int CPW = PIPE ? 8 : 1;                        // cells per wave
  static constexpr int WPB_ = 64 * 1024 / (STRIDE * 4);
  static constexpr int WPB = PIPE ? 1 : (WPB_ < 1 ? 1 : (WPB_ > 4 ? 4 : WPB_));  // waves per block
  // Cooperative form, for matrices of three or more row groups of which only one fits per
  // wave's LDS share: the four waves of a block share one cell's matrix, wave g forming
  // the rows of group g.
  static constexpr bool COOP = !PIPE && (NL + 63) / 64 >= 3 && WPB_ < 2;
  static constexpr int CPB = COOP ? 1 : WPB * CPW;  // cells per block
  static constexpr int THREADS = COOP ? 256 : 64 * WPB;
  static constexpr int LDS = (COOP ? 1 : WPB) * STRIDE * 4;
};

__device__ static inline void lds_dword(const void* gsrc, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_wave_base, 4, 0,
                                   0);
}

// Global node indices (component-major dofs) of the local rows lane + 64 rr of a cell.
template <int DIM, int P, int NCOMP, int NR, typename Pr>
__device__ static inline void cell_dofs(const Pr& pr, int cell, int lane, int64_t nodes[NR]) {
  constexpr int NP1 = P + 1;
  constexpr int NS = ipow(NP1, DIM);
  constexpr int NL = NCOMP * NS;
  const int cx = cell % pr.n[0];
  const int cy = (DIM >= 2) ? (cell / pr.n[0]) % pr.n[1] : 0;
  const int cz = (DIM == 3) ? cell / (pr.n[0] * pr.n[1]) : 0;
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    const int i = min(lane + 64 * rr, NL - 1);
    const int comp = i / NS, loc = i % NS;
    const int i0 = loc % NP1, i1 = (loc / NP1) % NP1, i2 = loc / (NP1 * NP1);
    nodes[rr] = (int64_t)comp * pr.nnodes + (cx * P + i0) +
                (int64_t)pr.np[0] * ((cy * P + i1) + (int64_t)pr.np[1] * (cz * P + i2));
  }
}

// y = K u for one cell from its packed upper triangle K and node values ue in LDS; lane
// i accumulates rows i, i + 64, ... in FP64 over the columns in order.  The entry (i, jj)
// sits at jj (jj + 1) / 2 + i when i <= jj and at i (i + 1) / 2 + jj otherwise; the column
// loop is split at 63 so that every row group for which all lanes take the same form
// skips the per-lane choice.
template <typename T, typename U, int NL, int NR>
__device__ static inline void cell_rows(const T* K, const U* ue, int lane, double y[NR]) {
  int row[NR], tri[NR];
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    y[rr] = 0.0;
    row[rr] = min(lane + 64 * rr, NL - 1);
    tri[rr] = row[rr] * (row[rr] + 1) / 2;
  }
  constexpr int JS = NL < 63 ? NL : 63;
  // columns 0 .. 62: rows of group 0 take either form, rows of later groups (>= 64) the
  // lower one
#pragma unroll 9
  for (int jj = 0; jj < JS; ++jj) {
    const double uj = (double)ue[jj];
    const int tj = jj * (jj + 1) / 2;
    y[0] += (double)K[(row[0] <= jj) ? tj + row[0] : tri[0] + jj] * uj;
#pragma unroll
    for (int rr = 1; rr < NR; ++rr) y[rr] += (double)K[tri[rr] + jj] * uj;
  }
  // columns 63 .. NL-1: rows of group 0 (<= 63) the upper form, later groups either
#pragma unroll 9
  for (int jj = JS; jj < NL; ++jj) {
    const double uj = (double)ue[jj];
    const int tj = jj * (jj + 1) / 2;
    y[0] += (double)K[tj + row[0]] * uj;
#pragma unroll
    for (int rr = 1; rr < NR; ++rr)
      y[rr] += (double)K[(row[rr] <= jj) ? tj + row[rr] : tri[rr] + jj] * uj;
  }
}

template <typename T, int DIM, int P, int NCOMP, bool SINGLE>
__global__ __launch_bounds__(256) void cut_apply_kernel(const CutProb<T>* __restrict__ probs,
                                                        int nprob, const CutProb<T> one,
                                                        int chunk, int j) {
  constexpr int NP1 = P + 1;
  constexpr int NS = ipow(NP1, DIM);
  constexpr int NL = NCOMP * NS;
  constexpr int NR = (NL + 63) / 64;
  using S = CutShape<T, NL>;
  extern __shared__ unsigned int lds_u32[];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  // neighbouring cut cells (neighbouring in space) on one XCD share node rows in its L2
  const int64_t blk = (int64_t)(blockIdx.x % 8) * chunk + (blockIdx.x / 8);
  int k = 0;
  if (!SINGLE) {
    int lo = 0, hi = nprob - 1;  // last record with blk0 <= blk
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (probs[mid].blk0 <= blk) lo = mid; else hi = mid - 1;
    }
    k = lo;
  }
  const CutProb<T>& pr = SINGLE ? one : probs[k];
  if (j >= pr.nsteps) return;
  const int64_t q0 = S::COOP ? blk - pr.blk0 : ((blk - pr.blk0) * S::WPB + wave) * S::CPW;
  if (q0 < 0 || q0 >= pr.ncand) return;
  const int ncell = (int)min((int64_t)S::CPW, pr.ncand - q0);

  unsigned int* kw = lds_u32 + (S::COOP ? 0 : wave) * S::STRIDE;
  const T* K = (const T*)kw;
  T* ue = (T*)(kw + S::KDP);
  const T* uin = ((pr.nsteps - 1 - j) & 1) ? pr.ua : pr.ub;
  const int64_t total = pr.ncand * S::KD;  // dwords of the packed array
  const unsigned int* kall = (const unsigned int*)pr.kcut;

  // the wave's cells (lane l holds cell q0 + l) and whether each is stepped (a cut cell
  // whose every leaf is void is reclassified and not stepped)
  int my_cell = 0, my_on = 0;
  if (lane < ncell) {
    my_cell = pr.cut_cells[q0 + lane];
    my_on = pr.info[my_cell] >= 0;
  }

  if constexpr (S::PIPE) {
    constexpr int KW = S::KDP / 64;
    double* ued = (double*)(kw + S::KDP);
    uint32_t kr[KW];
    T u0[NR];
    int64_t nodes[NR];
    // the loads of cell q: its matrix in whole 64-dword rows through a buffer resource
    // that ends at the array's end (reads past it return zero) and its node values of
    // rhs 0
    auto issue = [&](int64_t q, int cell) {
      const int64_t left = (total - q * S::KD) * 4;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(kall + q * S::KD), (short)0, (int)min(left, (int64_t)S::KDP * 4), 0x00020000);
#pragma unroll
      for (int w = 0; w < KW; ++w)
        kr[w] = __builtin_amdgcn_raw_buffer_load_b32(rs, (w * 64 + lane) * 4, 0, 0);
      cell_dofs<DIM, P, NCOMP, NR>(pr, cell, lane, nodes);
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) u0[rr] = uin[nodes[rr]];
    };
    issue(q0, __shfl(my_cell, 0));
    double yprev[NR];
    int64_t qprev = -1;
    for (int c = 0; c < ncell; ++c) {
      const int64_t q = q0 + c;
      const int on = __shfl(my_on, c);
      int64_t nd[NR];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) nd[rr] = nodes[rr];
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
      for (int w = 0; w < KW; ++w) kw[w * 64 + lane] = kr[w];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr)
        if (lane + 64 * rr < NL) ued[lane + 64 * rr] = (double)u0[rr];
      // the previous cell's rhs-0 products leave before the next loads are issued, so
      // the wait at the top of the next pass finds them done
      if (qprev >= 0) {
        T* yo = pr.y + qprev * NL;
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
          if (lane + 64 * rr < NL) yo[lane + 64 * rr] = (T)yprev[rr];
        qprev = -1;
      }
      if (c + 1 < ncell) issue(q + 1, __shfl(my_cell, c + 1));
      // LDS accesses of one wave complete in order; the barrier keeps the compiler's order
      __builtin_amdgcn_wave_barrier();
      if (on) {
        cell_rows<T, double, NL, NR>(K, ued, lane, yprev);
        qprev = q;
        // further right-hand sides: gathered and written here (not overlapped)
        for (int r = 1; r < pr.nrhs; ++r) {
          __builtin_amdgcn_wave_barrier();
          const T* u = uin + (int64_t)r * pr.ndof;
#pragma unroll
          for (int rr = 0; rr < NR; ++rr)
            if (lane + 64 * rr < NL) ued[lane + 64 * rr] = (double)u[nd[rr]];
          __builtin_amdgcn_wave_barrier();
          double yr[NR];
          cell_rows<T, double, NL, NR>(K, ued, lane, yr);
          T* yo = pr.y + ((int64_t)r * pr.ncand + q) * NL;
#pragma unroll
          for (int rr = 0; rr < NR; ++rr)
            if (lane + 64 * rr < NL) yo[lane + 64 * rr] = (T)yr[rr];
        }
      }
      // every lane has read this cell's LDS before the next pass overwrites it
      __builtin_amdgcn_wave_barrier();
    }
    if (qprev >= 0) {
      T* yo = pr.y + qprev * NL;
#pragma unroll
      for (int rr = 0; rr < NR; ++rr)
        if (lane + 64 * rr < NL) yo[lane + 64 * rr] = (T)yprev[rr];
    }
  } else if constexpr (S::COOP) {
    // one cell per block: the four waves bring its packed triangle global -> LDS by DMA,
    // wave 0 stages each right-hand side's node values, wave g < NR forms rows
    // lane + 64 g (columns in order, FP64 accumulation, as cell_rows)
    const int64_t q = q0;
    if (!__shfl(my_on, 0)) return;  // uniform over the block: one cell
    const int cell = __shfl(my_cell, 0);
    for (int w = wave; w < S::KDP / 64; w += 4)
      lds_dword(kall + min(q * S::KD + w * 64 + lane, total - 1), kw + w * 64);
    int64_t nodes[NR];
    cell_dofs<DIM, P, NCOMP, NR>(pr, cell, lane, nodes);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (pr.nrhs >= 2 && NL % 16 == 0) {
      // several right-hand sides: Y = K U on the matrix cores, 16 right-hand sides per
      // pass, wave w taking the row blocks w, w + 4, ... of 16 rows; A from the packed
      // triangle in LDS, B gathered from the node values of the pass's right-hand sides
      // (lane l16 + 16 k4 holds A[l16][k4] and B[k4][l16]; Mma<T>::row gives the result rows)
      constexpr int NMB = NL / 16, MPW = (NMB + 3) / 4;
      const int l16 = lane & 15, k4 = lane >> 4;
      const int cx = cell % pr.n[0], cy = (cell / pr.n[0]) % pr.n[1],
                cz = (DIM == 3) ? cell / (pr.n[0] * pr.n[1]) : 0;
      for (int r0 = 0; r0 < pr.nrhs; r0 += 16) {
        const int rr = r0 + l16;
        const bool rv = rr < pr.nrhs;
        const T* u = uin + (int64_t)(rv ? rr : 0) * pr.ndof;
        typename Mma<T>::acc acc[MPW];
#pragma unroll
        for (int m = 0; m < MPW; ++m)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[m][v] = 0;
        for (int ks = 0; ks < NL / 4; ++ks) {
          const int k = 4 * ks + k4;
          const int comp = k / NS, loc = k % NS;
          const int i0 = loc % NP1, i1 = (loc / NP1) % NP1, i2 = loc / (NP1 * NP1);
          const int64_t dof = (int64_t)comp * pr.nnodes + (cx * P + i0) +
                              (int64_t)pr.np[0] * ((cy * P + i1) + (int64_t)pr.np[1] * (cz * P + i2));
          const T bk = rv ? u[dof] : (T)0;
          const int tk = k * (k + 1) / 2;
#pragma unroll
          for (int m = 0; m < MPW; ++m) {
            const int mb = wave + 4 * m;
            if (mb < NMB) {
              const int i = mb * 16 + l16;
              acc[m] = Mma<T>::mma(K[(i <= k) ? tk + i : i * (i + 1) / 2 + k], bk, acc[m]);
            }
          }
        }
        if (rv) {
          T* yo = pr.y + ((int64_t)rr * pr.ncand + q) * NL;
#pragma unroll
          for (int m = 0; m < MPW; ++m) {
            const int mb = wave + 4 * m;
            if (mb < NMB)
#pragma unroll
              for (int v = 0; v < 4; ++v) yo[mb * 16 + Mma<T>::row(k4, v)] = (T)acc[m][v];
          }
        }
      }
      return;
    }
    const int row = lane + 64 * wave;
    const int tr = row * (row + 1) / 2;
    for (int r = 0; r < pr.nrhs; ++r) {
      const T* u = uin + (int64_t)r * pr.ndof;
      if (wave == 0) {
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
          if (lane + 64 * rr < NL) ue[lane + 64 * rr] = u[nodes[rr]];
      }
      __syncthreads();
      if (wave < NR && row < NL) {
        double y = 0.0;
#pragma unroll 8
        for (int jj = 0; jj < NL; ++jj)
          y += (double)K[(row <= jj) ? jj * (jj + 1) / 2 + row : tr + jj] * (double)ue[jj];
        pr.y[((int64_t)r * pr.ncand + q) * NL + row] = (T)y;
      }
      // every wave has read ue before the next right-hand side overwrites it
      __syncthreads();
    }
  } else {
    // one cell per wave: packed triangle global -> LDS by DMA (64 coalesced dwords per
    // instruction, no registers), node values of rhs 0 in flight alongside
    const int64_t q = q0;
    if (!__shfl(my_on, 0)) return;
    const int cell = __shfl(my_cell, 0);
#pragma unroll 4
    for (int w = 0; w < S::KDP / 64; ++w)
      lds_dword(kall + min(q * S::KD + w * 64 + lane, total - 1), kw + w * 64);
    int64_t nodes[NR];
    cell_dofs<DIM, P, NCOMP, NR>(pr, cell, lane, nodes);
    T u0[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) u0[rr] = uin[nodes[rr]];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    for (int r = 0; r < pr.nrhs; ++r) {
      const T* u = uin + (int64_t)r * pr.ndof;
#pragma unroll
      for (int rr = 0; rr < NR; ++rr)
        if (lane + 64 * rr < NL) ue[lane + 64 * rr] = (r == 0) ? u0[rr] : u[nodes[rr]];
      __builtin_amdgcn_wave_barrier();
      double y[NR];
      cell_rows<T, T, NL, NR>(K, ue, lane, y);
      T* yo = pr.y + ((int64_t)r * pr.ncand + q) * NL;
#pragma unroll
      for (int rr = 0; rr < NR; ++rr)
        if (lane + 64 * rr < NL) yo[lane + 64 * rr] = (T)y[rr];
      // every lane has read ue before the next right-hand side overwrites it
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <typename T, int DIM, int P, int NCOMP>
struct CutKind {
  static constexpr int NL = NCOMP * ipow(P + 1, DIM);
  using S = CutShape<T, NL>;
  static fcw_status launch(hipStream_t s, const void* probs, int nprob, const void* one,
                           int64_t nblk, int j) {
    if (nblk <= 0) return FCW_OK;
    const int chunk = (int)((nblk + 7) / 8);
    if (one) {
      CutProb<T> rec;
      std::memcpy(&rec, one, sizeof rec);
      auto kern = cut_apply_kernel<T, DIM, P, NCOMP, true>;
      // set once (not a stream operation, so also safe while a graph is being captured)
      static const hipError_t attr = hipFuncSetAttribute(
          (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS);
      FCW_HIP(attr);
      kern<<<(unsigned)(8 * chunk), S::THREADS, S::LDS, s>>>(nullptr, 1, rec, chunk, j);
    } else {
      auto kern = cut_apply_kernel<T, DIM, P, NCOMP, false>;
      static const hipError_t attr = hipFuncSetAttribute(
          (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS);
      FCW_HIP(attr);
      kern<<<(unsigned)(8 * chunk), S::THREADS, S::LDS, s>>>((const CutProb<T>*)probs, nprob,
                                                              CutProb<T>{}, chunk, j);
    }
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
};

using CutLaunch = fcw_status (*)(hipStream_t, const void*, int, const void*, int64_t, int);

// launcher and cells per block of the cut-cell kernel of a problem kind (null if not built)
static CutLaunch cut_kind(const Ctx& c, int* cpb) {
  const bool f64 = c.precision == FCW_FP64;
#define FCW_CUT(D, PP, NC)                                                          \
  if (c.dim == D && c.p == PP && c.ncomp == NC) {                                   \
    if (f64) { *cpb = CutKind<double, D, PP, NC>::S::CPB; return &CutKind<double, D, PP, NC>::launch; } \
    *cpb = CutKind<float, D, PP, NC>::S::CPB;                                        \
    return &CutKind<float, D, PP, NC>::launch;                                       \
  }
  FCW_CUT(2, 1, 1) FCW_CUT(2, 2, 1) FCW_CUT(2, 3, 1) FCW_CUT(2, 4, 1) FCW_CUT(2, 5, 1)
  FCW_CUT(2, 6, 1)
  FCW_CUT(3, 1, 1) FCW_CUT(3, 2, 1) FCW_CUT(3, 3, 1) FCW_CUT(3, 4, 1)
  FCW_CUT(3, 1, 3) FCW_CUT(3, 2, 3) FCW_CUT(3, 3, 3)
#undef FCW_CUT
  return nullptr;
}

static_assert(sizeof(CutProb<double>) <= 256 && sizeof(CutProb<float>) == sizeof(CutProb<double>),
              "callers hold a record in 256 bytes");

size_t cutprob_size(int fp64) { return fp64 ? sizeof(CutProb<double>) : sizeof(CutProb<float>); }

// Allocate the products buffer for nrhs right-hand sides (kept and grown on demand).
fcw_status ensure_ycut(Ctx& c, int nrhs) {
  const size_t bytes = (size_t)nrhs * c.n_cut_cand * c.n_loc * c.state_bytes();
  if (c.ycut_bytes >= bytes) return FCW_OK;
  if (c.d_ycut) FCW_HIP(hipFree(c.d_ycut));
  c.footprint -= (int64_t)c.ycut_bytes;
  c.d_ycut = nullptr;
  c.ycut_bytes = 0;
  if (bytes == 0) return FCW_OK;
  FCW_HIP(hipMalloc(&c.d_ycut, bytes));
  c.ycut_bytes = bytes;
  c.footprint += (int64_t)bytes;
  return FCW_OK;
}

template <typename T>
static void fill(const Ctx& c, void* out, const void* ua, const void* ub, int nrhs, int nsteps,
                 int64_t blk0) {
  CutProb<T> p{};
  p.ua = (const T*)ua;
  p.ub = (const T*)ub;
  p.kcut = (const T*)c.d_kcut_s;
  p.cut_cells = c.d_cut_cells;
  p.info = c.d_info;
  p.y = (T*)c.d_ycut;
  p.ncand = c.n_cut_cand;
  p.nnodes = c.nnodes;
  p.ndof = c.ndof;
  p.blk0 = blk0;
  for (int k = 0; k < 3; ++k) {
    p.n[k] = (k < c.dim) ? c.ncells[k] : 1;
    p.np[k] = (k < c.dim) ? c.npts[k] : 1;
  }
  p.nrhs = nrhs;
  p.nsteps = nsteps;
  std::memcpy(out, &p, sizeof p);
}

// Record of one problem for the cut-cell kernel (ensure_ycut must have run for nrhs);
// returns the number of blocks the problem takes.
int64_t cutprob_fill(const Ctx& c, void* out, const void* ua, const void* ub, int nrhs,
                     int nsteps, int64_t blk0) {
  int cpb = 1;
  if (!cut_kind(c, &cpb)) cpb = 1;
  if (c.precision == FCW_FP64) fill<double>(c, out, ua, ub, nrhs, nsteps, blk0);
  else fill<float>(c, out, ua, ub, nrhs, nsteps, blk0);
  return (c.n_cut_cand + cpb - 1) / cpb;
}

// One launch of the cut-cell kernel: a single record by value (`one`), or nprob device
// records covering nblk blocks; step j of the call.
fcw_status launch_cut(const Ctx& kind, hipStream_t s, const void* probs, int nprob,
                      const void* one, int64_t nblk, int j) {
  int cpb = 1;
  CutLaunch f = cut_kind(kind, &cpb);
  if (!f) {
    set_error("cut-cell kernel not built for dim=%d p=%d ncomp=%d", kind.dim, kind.p, kind.ncomp);
    return FCW_E_UNSUPPORTED;
  }
  return f(s, probs, nprob, one, nblk, j);
}

// y_cut = K_e u for every cut cell of one problem and right-hand side.
fcw_status launch_cut_products(Ctx& c, int nrhs, const void* u) {
  if (c.n_cut_cand == 0) return FCW_OK;
  fcw_status st = ensure_ycut(c, nrhs);
  if (st) return st;
  char rec[sizeof(CutProb<double>)];
  const int64_t nblk = cutprob_fill(c, rec, u, u, nrhs, 1, 0);
  return launch_cut(c, c.stream, nullptr, 1, rec, nblk, 0);
}

}  // namespace fcw
