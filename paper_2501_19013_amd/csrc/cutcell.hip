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
  static constexpr int KD = NL * (NL + 1) / 2 * (int)(sizeof(T) / 4);  // dwords per matrix
  static constexpr int KDP = (KD + 63) / 64 * 64;
  static constexpr int UEP = (NL * (int)(sizeof(T) / 4) + 63) / 64 * 64;
  static constexpr int STRIDE = KDP + UEP;  // LDS dwords per wave
  static constexpr int WPB_ = 64 * 1024 / (STRIDE * 4);
  static constexpr int WPB = WPB_ < 1 ? 1 : (WPB_ > 4 ? 4 : WPB_);  // waves per block
  static constexpr int LDS = WPB * STRIDE * 4;
};

__device__ static inline void lds_dword(const void* gsrc, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_wave_base, 4, 0,
                                   0);
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

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
  const int64_t q = (blk - pr.blk0) * S::WPB + wave;
  if (q < 0 || q >= pr.ncand) return;
  const int cell = pr.cut_cells[q];
  if (pr.info[cell] < 0) return;  // reclassified (every leaf void): not stepped

  unsigned int* kw = lds_u32 + wave * S::STRIDE;
  const T* K = (const T*)kw;
  T* ue = (T*)(kw + S::KDP);
  const unsigned int* src = (const unsigned int*)pr.kcut + q * S::KD;
  const int64_t rem = (pr.ncand - q) * S::KD;  // dwords of the array from this matrix on
#pragma unroll 4
  for (int w = 0; w < S::KDP / 64; ++w) {
    const int64_t o = min((int64_t)(w * 64 + lane), rem - 1);
    lds_dword(src + o, kw + w * 64);
  }
  const int cx = cell % pr.n[0];
  const int cy = (DIM >= 2) ? (cell / pr.n[0]) % pr.n[1] : 0;
  const int cz = (DIM == 3) ? cell / (pr.n[0] * pr.n[1]) : 0;
  int64_t nodes[NR];
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    const int i = min(lane + 64 * rr, NL - 1);
    const int comp = i / NS, loc = i % NS;
    const int i0 = loc % NP1, i1 = (loc / NP1) % NP1, i2 = loc / (NP1 * NP1);
    nodes[rr] = (int64_t)comp * pr.nnodes + (cx * P + i0) +
                (int64_t)pr.np[0] * ((cy * P + i1) + (int64_t)pr.np[1] * (cz * P + i2));
  }
  const T* uin = ((pr.nsteps - 1 - j) & 1) ? pr.ua : pr.ub;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

  for (int r = 0; r < pr.nrhs; ++r) {
    const T* u = uin + (int64_t)r * pr.ndof;
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      const int i = lane + 64 * rr;
      if (i < NL) ue[i] = u[nodes[rr]];
    }
    // LDS accesses of one wave complete in order; the barrier keeps the compiler's order
    __builtin_amdgcn_wave_barrier();
    double y[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) y[rr] = 0.0;
#pragma unroll 9
    for (int jj = 0; jj < NL; ++jj) {
      const double uj = (double)ue[jj];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) {
        const int i = min(lane + 64 * rr, NL - 1);
        const int idx = (i <= jj) ? jj * (jj + 1) / 2 + i : i * (i + 1) / 2 + jj;
        y[rr] += (double)K[idx] * uj;
      }
    }
    T* yo = pr.y + ((int64_t)r * pr.ncand + q) * NL;
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      const int i = lane + 64 * rr;
      if (i < NL) yo[i] = (T)y[rr];
    }
    // every lane has read ue before the next right-hand side overwrites it
    __builtin_amdgcn_wave_barrier();
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
      kern<<<(unsigned)(8 * chunk), 64 * S::WPB, S::LDS, s>>>(nullptr, 1, rec, chunk, j);
    } else {
      auto kern = cut_apply_kernel<T, DIM, P, NCOMP, false>;
      static const hipError_t attr = hipFuncSetAttribute(
          (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS);
      FCW_HIP(attr);
      kern<<<(unsigned)(8 * chunk), 64 * S::WPB, S::LDS, s>>>((const CutProb<T>*)probs, nprob,
                                                              CutProb<T>{}, chunk, j);
    }
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
};

using CutLaunch = fcw_status (*)(hipStream_t, const void*, int, const void*, int64_t, int);

// launcher and waves per block of the cut-cell kernel of a problem kind (null if not built)
static CutLaunch cut_kind(const Ctx& c, int* wpb) {
  const bool f64 = c.precision == FCW_FP64;
#define FCW_CUT(D, PP, NC)                                                          \
  if (c.dim == D && c.p == PP && c.ncomp == NC) {                                   \
    if (f64) { *wpb = CutKind<double, D, PP, NC>::S::WPB; return &CutKind<double, D, PP, NC>::launch; } \
    *wpb = CutKind<float, D, PP, NC>::S::WPB;                                        \
    return &CutKind<float, D, PP, NC>::launch;                                       \
  }
  FCW_CUT(2, 1, 1) FCW_CUT(2, 2, 1) FCW_CUT(2, 3, 1) FCW_CUT(2, 4, 1) FCW_CUT(2, 5, 1)
  FCW_CUT(2, 6, 1)
  FCW_CUT(3, 1, 1) FCW_CUT(3, 2, 1) FCW_CUT(3, 3, 1) FCW_CUT(3, 4, 1)
  FCW_CUT(3, 1, 3) FCW_CUT(3, 2, 3)
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
  int wpb = 1;
  if (!cut_kind(c, &wpb)) wpb = 1;
  if (c.precision == FCW_FP64) fill<double>(c, out, ua, ub, nrhs, nsteps, blk0);
  else fill<float>(c, out, ua, ub, nrhs, nsteps, blk0);
  return (c.n_cut_cand + wpb - 1) / wpb;
}

// One launch of the cut-cell kernel: a single record by value (`one`), or nprob device
// records covering nblk blocks; step j of the call.
fcw_status launch_cut(const Ctx& kind, hipStream_t s, const void* probs, int nprob,
                      const void* one, int64_t nblk, int j) {
  int wpb = 1;
  CutLaunch f = cut_kind(kind, &wpb);
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
