// The explicit step of the spectral cell method on gfx950: one fused tile kernel per
// central-difference step (paper eq. cdm), organised for CDNA4:
//
//  * A workgroup (4 wave64) owns a tile of TX x TY (x TZ) cells and every node in the
//    half-open node box of those cells.  It stages the node values of the tile plus
//    one ring of cells on the low side in LDS (coalesced row loads), so each owned
//    node sees every cell around it without atomics or a second pass.
//  * Uncut cells share the reference stiffness K_ref (Sec. 2.2): their products are
//    one batched dense contraction Y = K_ref [u_e1 ... u_e16] on the matrix cores
//    (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64), K_ref rows as the A operand,
//    16 cells as the B operand gathered from the LDS node tile.
//  * Cut cells stream their own stiffness K_e, packed upper triangle, from HBM;
//    one wave per cell, lanes = rows.
//  * Element results land in LDS; each owned node gathers them from its (at most
//    2^d) cells in a fixed order (atomic-free, bitwise reproducible) and applies the
//    lumped-mass update in increment form
//        d_{k+1} = d_k + dt^2 M^{-1} (F_k - K u_k),  u_{k+1} = u_k + d_{k+1},
//    which is eq. cdm with d_k = u_k - u_{k-1}; the first step of a run uses half
//    the acceleration (Alg. newmark with beta = 0).
//  * Tiles are mapped to blocks XCD by XCD (blocks b, b+8, ... run on one XCD and get
//    neighbouring tiles, so halo rows are shared through that XCD's L2).
#include <cmath>

#include "common.h"

namespace fcw {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
// Lane layouts (16x16x4, one block): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
// the output D[i][j] sits in lane j + 16 * (i / 4), item i % 4 for f32 and in lane
// j + 16 * (i % 4), item i / 4 for f64.
template <>
struct Mma<float> {
  using acc = f32x4;
  __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
  __device__ static inline acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<double> {
  using acc = f64x4;
  __device__ static inline int row(int lk, int r) { return 4 * r + lk; }
  __device__ static inline acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

enum { kModeStep = 0, kModeApply = 1, kModeLanczos = 2 };

template <typename T>
struct StepArgs {
  const T* u_in;
  T* u_out;
  T* d;
  const T* invm;
  const double* invm64;
  const int32_t* info;
  const T* kref;
  const T* kcut;
  int n[3], np[3], ntile[3];
  int ntiles, chunk;
  int64_t nnodes, ndof;
  T dt2;
  int start;
  const SourceDev* src;
  double t;
};

__device__ static inline double ricker(double t, double f0) {
  const double pi = 3.14159265358979323846;
  const double ts = 2.0 * sqrt(6.0) / (pi * f0);
  const double q = pi * f0 * (t - ts);
  return (1.0 - 2.0 * q * q) * exp(-q * q);
}

template <typename T, int DIM, int P, int NCOMP, int TX, int TY, int TZ, int MODE>
__global__ __launch_bounds__(256) void tile_kernel(StepArgs<T> a) {
  constexpr int NP1 = P + 1;
  constexpr int NS = ipow(NP1, DIM);
  constexpr int NL = NCOMP * NS;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  constexpr int KW = NKS * 4;
  constexpr int RCX = TX + 1;
  constexpr int RCY = (DIM >= 2) ? TY + 1 : 1;
  constexpr int RCZ = (DIM == 3) ? TZ + 1 : 1;
  constexpr int NRC = RCX * RCY * RCZ;
  constexpr int RNX = RCX * P + 1;
  constexpr int RNY = (DIM >= 2) ? RCY * P + 1 : 1;
  constexpr int RNZ = (DIM == 3) ? RCZ * P + 1 : 1;
  constexpr int NRN = RNX * RNY * RNZ;
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr bool AREG = NMB * NKS <= 32;  // keep K_ref fragments in VGPRs
  // otherwise stage them in LDS when small enough, else read them through the caches
  constexpr bool ALDS = !AREG && (NMB * 16 * KW * (int)sizeof(T) <= 48 * 1024);
  constexpr int NB = (NRC + 15) / 16;

  __shared__ T u_s[NCOMP * NRN];
  __shared__ T y_s[NRC * NL];
  __shared__ T a_s[ALDS ? NMB * 16 * KW : 1];
  __shared__ int info_s[NRC];
  __shared__ int off_s[KW];
  __shared__ double ft_s;
  __shared__ int src_on;

  const int tile = (int)(blockIdx.x % 8) * a.chunk + (int)(blockIdx.x / 8);
  if (tile >= a.ntiles) return;
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x;
  const int tx = tile % a.ntile[0];
  const int ty = (DIM >= 2) ? (tile / a.ntile[0]) % a.ntile[1] : 0;
  const int tz = (DIM == 3) ? tile / (a.ntile[0] * a.ntile[1]) : 0;
  const int cx0 = tx * TX, cy0 = ty * TY, cz0 = tz * TZ;
  const int rcx0 = cx0 - 1;
  const int rcy0 = (DIM >= 2) ? cy0 - 1 : 0;
  const int rcz0 = (DIM == 3) ? cz0 - 1 : 0;
  const int rnx0 = rcx0 * P, rny0 = rcy0 * P, rnz0 = rcz0 * P;
  const T* uin = a.u_in + (int64_t)rhs * a.ndof;

  // ---- stage cell info, node values, K_ref, local offsets ----
  for (int c = tid; c < NRC; c += 256) {
    const int lx = c % RCX, ly = (c / RCX) % RCY, lz = c / (RCX * RCY);
    const int gx = rcx0 + lx, gy = rcy0 + ly, gz = rcz0 + lz;
    int v = kInfoOut;
    if (gx >= 0 && gx < a.n[0] && gy >= 0 && gy < a.n[1] && gz >= 0 && gz < a.n[2])
      v = a.info[gx + (int64_t)a.n[0] * (gy + (int64_t)a.n[1] * gz)];
    info_s[c] = v;
  }
  for (int comp = 0; comp < NCOMP; ++comp) {
    const T* uc = uin + (int64_t)comp * a.nnodes;
    for (int i = tid; i < NRN; i += 256) {
      const int lx = i % RNX, ly = (i / RNX) % RNY, lz = i / (RNX * RNY);
      const int gx = rnx0 + lx, gy = rny0 + ly, gz = rnz0 + lz;
      T v = T(0);
      if (gx >= 0 && gx < a.np[0] && gy >= 0 && gy < a.np[1] && gz >= 0 && gz < a.np[2]) {
        const int64_t node = gx + (int64_t)a.np[0] * (gy + (int64_t)a.np[1] * gz);
        v = uc[node];
        if (MODE == kModeLanczos) v = v * (T)sqrt(a.invm64[node]);
      }
      u_s[comp * NRN + i] = v;
    }
  }
  if (ALDS) {
    for (int i = tid; i < NMB * 16 * KW; i += 256) {
      const int r = i / KW, cc = i % KW;
      a_s[i] = (r < NL && cc < NL) ? a.kref[r * NL + cc] : T(0);
    }
  }
  for (int j = tid; j < KW; j += 256) {
    int off = -1;
    if (j < NL) {
      const int comp = j / NS, loc = j % NS;
      const int i0 = loc % NP1, i1 = (loc / NP1) % NP1, i2 = loc / (NP1 * NP1);
      off = comp * NRN + i0 + RNX * (i1 + RNY * i2);
    }
    off_s[j] = off;
  }
  if (tid == 0) {
    src_on = 0;
    ft_s = 0.0;
    if (MODE == kModeStep && a.src != nullptr) {
      const SourceDev& s = a.src[rhs];
      // owned node box of this tile vs node box of the source cell
      bool hit = true;
      const int c0[3] = {cx0, cy0, cz0};
      const int tt[3] = {TX, TY, TZ};
      for (int k = 0; k < DIM; ++k) {
        const int o0 = c0[k] * P;
        const int o1 = (c0[k] + tt[k] >= a.n[k]) ? a.np[k] : (c0[k] + tt[k]) * P;
        const int s0 = s.cell[k] * P, s1 = s.cell[k] * P + P;
        if (s1 < o0 || s0 >= o1) hit = false;
      }
      if (hit) {
        src_on = 1;
        ft_s = ricker(a.t, s.f0);
      }
    }
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;

  // ---- uncut cells: batched K_ref contraction on the matrix cores ----
  {
    int offk[NKS];
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) offk[kk] = off_s[4 * kk + lk];
    T areg[AREG ? NMB : 1][AREG ? NKS : 1];
    if (AREG) {
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int kk = 0; kk < NKS; ++kk) {
          const int r = mb * 16 + lc, cc = 4 * kk + lk;
          areg[AREG ? mb : 0][AREG ? kk : 0] = (r < NL && cc < NL) ? a.kref[r * NL + cc] : T(0);
        }
    }
    for (int b = wave; b < NB; b += 4) {
      const int c = b * 16 + lc;
      const bool valid = (c < NRC) && (info_s[c] == kInfoUncut);
      int base = 0;
      if (c < NRC) {
        const int lx = c % RCX, ly = (c / RCX) % RCY, lz = c / (RCX * RCY);
        base = lx * P + RNX * (ly * P + RNY * (lz * P));
      }
      typename Mma<T>::acc acc[NMB];
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) acc[mb] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk) {
        const T bv = (valid && offk[kk] >= 0) ? u_s[base + offk[kk]] : T(0);
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          T av;
          if (AREG) {
            av = areg[AREG ? mb : 0][AREG ? kk : 0];
          } else if (ALDS) {
            av = a_s[ALDS ? (mb * 16 + lc) * KW + 4 * kk + lk : 0];
          } else {
            const int r = mb * 16 + lc, cc = 4 * kk + lk;
            av = (r < NL && cc < NL) ? a.kref[r * NL + cc] : T(0);
          }
          acc[mb] = Mma<T>::mma(av, bv, acc[mb]);
        }
      }
      if (valid) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = mb * 16 + Mma<T>::row(lk, r);
            if (i < NL) y_s[c * NL + i] = acc[mb][r];
          }
      }
    }
  }

  // ---- cut cells: own packed stiffness streamed from HBM, one wave per cell ----
  {
    int seen = 0;
    for (int c0 = 0; c0 < NRC; c0 += 64) {
      const int cc = c0 + lane;
      const bool isc = (cc < NRC) && (info_s[cc] >= 0);
      unsigned long long mask = __ballot(isc);
      while (mask) {
        const int bit = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        if ((seen++ & 3) != wave) continue;
        const int c = c0 + bit;
        const int q = info_s[c];
        const int lx = c % RCX, ly = (c / RCX) % RCY, lz = c / (RCX * RCY);
        const int base = lx * P + RNX * (ly * P + RNY * (lz * P));
        // the FP64 Lanczos operator reads the full FP64 setup matrices
        const T* K = a.kcut + (int64_t)q * (MODE == kModeLanczos ? NL * NL : NPK);
        for (int i = lane; i < NL; i += 64) {
          T y = T(0);
          for (int j = 0; j < NL; ++j) {
            const int idx = (MODE == kModeLanczos)
                                ? i * NL + j
                                : ((i <= j) ? j * (j + 1) / 2 + i : i * (i + 1) / 2 + j);
            y += K[idx] * u_s[base + off_s[j]];
          }
          y_s[c * NL + i] = y;
        }
      }
    }
  }
  __syncthreads();

  // ---- owned nodes: fixed-order gather of element results + update ----
  const int ox0 = cx0 * P;
  const int ox1 = (cx0 + TX >= a.n[0]) ? a.np[0] : (cx0 + TX) * P;
  const int oy0 = (DIM >= 2) ? cy0 * P : 0;
  const int oy1 = (DIM >= 2) ? ((cy0 + TY >= a.n[1]) ? a.np[1] : (cy0 + TY) * P) : 1;
  const int oz0 = (DIM == 3) ? cz0 * P : 0;
  const int oz1 = (DIM == 3) ? ((cz0 + TZ >= a.n[2]) ? a.np[2] : (cz0 + TZ) * P) : 1;
  const int onx = ox1 - ox0, ony = oy1 - oy0, onz = oz1 - oz0;
  const int nown = onx * ony * onz;
  for (int i = tid; i < nown; i += 256) {
    const int gx = ox0 + i % onx;
    const int gy = oy0 + (i / onx) % ony;
    const int gz = oz0 + i / (onx * ony);
    const int64_t node = gx + (int64_t)a.np[0] * (gy + (int64_t)a.np[1] * gz);
    int cl[3], ch[3];
    const int g3[3] = {gx, gy, gz};
    for (int k = 0; k < 3; ++k) {
      if (k >= DIM) { cl[k] = ch[k] = 0; continue; }
      int hi = g3[k] / P;
      int lo = (g3[k] % P == 0) ? hi - 1 : hi;
      if (hi > a.n[k] - 1) hi = a.n[k] - 1;
      if (lo < 0) lo = 0;
      cl[k] = lo;
      ch[k] = hi;
    }
    T r[NCOMP];
#pragma unroll
    for (int comp = 0; comp < NCOMP; ++comp) r[comp] = T(0);
    for (int cz = cl[2]; cz <= ch[2]; ++cz)
      for (int cy = cl[1]; cy <= ch[1]; ++cy)
        for (int cx = cl[0]; cx <= ch[0]; ++cx) {
          const int lcell = (cx - rcx0) + RCX * ((cy - rcy0) + RCY * (cz - rcz0));
          if (info_s[lcell] == kInfoOut) continue;
          const int loc = (gx - cx * P) + NP1 * ((gy - cy * P) + NP1 * (gz - cz * P));
#pragma unroll
          for (int comp = 0; comp < NCOMP; ++comp) r[comp] += y_s[lcell * NL + comp * NS + loc];
        }
    if (MODE == kModeStep) {
      const int rl = (gx - rnx0) + RNX * ((gy - rny0) + RNY * (gz - rnz0));
      const T im = a.invm[node];
      int sloc = -1;
      if (src_on) {
        const SourceDev& s = a.src[rhs];
        const int sx = gx - s.cell[0] * P, sy = gy - s.cell[1] * P, sz = gz - s.cell[2] * P;
        if (sx >= 0 && sx <= P && (DIM < 2 || (sy >= 0 && sy <= P)) &&
            (DIM < 3 || (sz >= 0 && sz <= P)))
          sloc = sx + NP1 * ((DIM >= 2 ? sy : 0) + NP1 * (DIM == 3 ? sz : 0));
      }
#pragma unroll
      for (int comp = 0; comp < NCOMP; ++comp) {
        const int64_t dof = (int64_t)rhs * a.ndof + (int64_t)comp * a.nnodes + node;
        T F = T(0);
        if (sloc >= 0) F = (T)(ft_s * a.src[rhs].b[comp * NS + sloc]);
        T acc = a.dt2 * im * (F - r[comp]);
        if (a.start) acc = acc * T(0.5);
        const T dn = a.d[dof] + acc;
        a.d[dof] = dn;
        a.u_out[dof] = u_s[comp * NRN + rl] + dn;
      }
    } else if (MODE == kModeApply) {
#pragma unroll
      for (int comp = 0; comp < NCOMP; ++comp)
        a.u_out[(int64_t)rhs * a.ndof + (int64_t)comp * a.nnodes + node] = r[comp];
    } else {
      const T s = (T)sqrt(a.invm64[node]);
#pragma unroll
      for (int comp = 0; comp < NCOMP; ++comp)
        a.u_out[(int64_t)comp * a.nnodes + node] = s * r[comp];
    }
  }
}

// --------------------------------------------------------------------------------
// dispatch
// --------------------------------------------------------------------------------

template <typename T>
static StepArgs<T> make_args(const Ctx& c, int tx, int ty, int tz) {
  StepArgs<T> a{};
  a.info = c.d_info;
  a.kref = (const T*)c.d_kref_s;
  a.kcut = (const T*)c.d_kcut_s;
  a.invm = (const T*)c.d_invm;
  a.invm64 = c.d_invm64;
  const int tt[3] = {tx, ty, tz};
  a.ntiles = 1;
  for (int k = 0; k < 3; ++k) {
    a.n[k] = (k < c.dim) ? c.ncells[k] : 1;
    a.np[k] = (k < c.dim) ? c.npts[k] : 1;
    a.ntile[k] = (k < c.dim) ? (a.n[k] + tt[k] - 1) / tt[k] : 1;
    a.ntiles *= a.ntile[k];
  }
  a.chunk = (a.ntiles + 7) / 8;
  a.nnodes = c.nnodes;
  a.ndof = c.ndof;
  return a;
}

template <typename T, int DIM, int P, int NCOMP, int TX, int TY, int TZ>
struct TileCfg {
  static fcw_status run(Ctx& c, int mode, int nrhs, const void* uin, void* uout, void* d,
                        double t, double dt, int start) {
    StepArgs<T> a = make_args<T>(c, TX, TY, TZ);
    a.u_in = (const T*)uin;
    a.u_out = (T*)uout;
    a.d = (T*)d;
    a.dt2 = (T)(dt * dt);
    a.start = start;
    a.src = (mode == kModeStep) ? c.d_src : nullptr;
    a.t = t;
    if (mode == kModeLanczos) {
      a.kref = (const T*)c.d_kref;
      a.kcut = (const T*)c.d_kcut;
    }
    dim3 grid(8 * a.chunk, nrhs, 1);
    if (mode == kModeStep)
      tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeStep><<<grid, 256, 0, c.stream>>>(a);
    else if (mode == kModeApply)
      tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeApply><<<grid, 256, 0, c.stream>>>(a);
    else
      tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeLanczos><<<grid, 256, 0, c.stream>>>(a);
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
};

using RunFn = fcw_status (*)(Ctx&, int, int, const void*, void*, void*, double, double, int);

template <typename T>
static RunFn select_kernel(const Ctx& c) {
  constexpr bool F64 = sizeof(T) == 8;
#define FCW_CASE(D, PP, NC, TX, TY, TZ)                        \
  if (c.dim == D && c.p == PP && c.ncomp == NC)                \
    return &TileCfg<T, D, PP, NC, TX, TY, TZ>::run;
  if constexpr (F64) {
    FCW_CASE(2, 1, 1, 32, 16, 1) FCW_CASE(2, 2, 1, 16, 16, 1) FCW_CASE(2, 3, 1, 16, 8, 1)
    FCW_CASE(2, 4, 1, 16, 8, 1) FCW_CASE(2, 5, 1, 8, 8, 1) FCW_CASE(2, 6, 1, 8, 8, 1)
    FCW_CASE(3, 1, 1, 8, 8, 4) FCW_CASE(3, 2, 1, 8, 4, 4) FCW_CASE(3, 3, 1, 4, 4, 4)
    FCW_CASE(3, 4, 1, 4, 4, 2)
    FCW_CASE(3, 1, 3, 8, 4, 4) FCW_CASE(3, 2, 3, 4, 4, 2)
  } else {
    FCW_CASE(2, 1, 1, 32, 32, 1) FCW_CASE(2, 2, 1, 16, 16, 1) FCW_CASE(2, 3, 1, 16, 16, 1)
    FCW_CASE(2, 4, 1, 16, 16, 1) FCW_CASE(2, 5, 1, 16, 8, 1) FCW_CASE(2, 6, 1, 8, 8, 1)
    FCW_CASE(3, 1, 1, 8, 8, 8) FCW_CASE(3, 2, 1, 8, 4, 4) FCW_CASE(3, 3, 1, 4, 4, 4)
    FCW_CASE(3, 4, 1, 4, 4, 2)
    FCW_CASE(3, 1, 3, 8, 4, 4) FCW_CASE(3, 2, 3, 4, 4, 4)
  }
#undef FCW_CASE
  return nullptr;
}

static RunFn select_for(const Ctx& c, bool fp64) {
  return fp64 ? select_kernel<double>(c) : select_kernel<float>(c);
}

bool step_supported(const Ctx& c) {
  return select_for(c, c.precision == FCW_FP64) != nullptr && select_for(c, true) != nullptr;
}

fcw_status launch_step(Ctx& c, int nrhs, const void* u_in, void* u_out, void* d, double t,
                       double dt, int start) {
  RunFn f = select_for(c, c.precision == FCW_FP64);
  if (!f) {
    set_error("step kernel not built for dim=%d p=%d ncomp=%d", c.dim, c.p, c.ncomp);
    return FCW_E_UNSUPPORTED;
  }
  return f(c, kModeStep, nrhs, u_in, u_out, d, t, dt, start);
}

fcw_status launch_apply(Ctx& c, int nrhs, const void* u, void* r) {
  RunFn f = select_for(c, c.precision == FCW_FP64);
  if (!f) {
    set_error("stiffness kernel not built for dim=%d p=%d ncomp=%d", c.dim, c.p, c.ncomp);
    return FCW_E_UNSUPPORTED;
  }
  return f(c, kModeApply, nrhs, u, r, nullptr, 0.0, 0.0, 0);
}

// w = M^{-1/2} K M^{-1/2} v in FP64 (uses the FP64 operands held for the Lanczos solve)
fcw_status launch_apply_scaled64(Ctx& c, const double* v, double* w) {
  RunFn f = select_for(c, true);
  if (!f) {
    set_error("FP64 stiffness kernel not built for dim=%d p=%d ncomp=%d", c.dim, c.p, c.ncomp);
    return FCW_E_UNSUPPORTED;
  }
  return f(c, kModeLanczos, 1, v, w, nullptr, 0.0, 0.0, 0);
}

}  // namespace fcw
