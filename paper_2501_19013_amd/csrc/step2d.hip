// Central-difference step (paper eq. cdm) for 2-D scalar problems, shaped for CDNA4 wave64.
// One launch advances every item of a work list -- (problem, right-hand side, tile) --
// by one step, so several problems of one kind (same p and precision; any size,
// geometry and sources) and many right-hand sides share a launch.
//
//  * A tile is TX = 64 / P cells wide, so one owned node row of a tile is exactly one
//    wave (lane = x); TY cells high.  A workgroup (4 waves) stages the node values of
//    the tile plus one ring of cells on the low side in LDS, one region row per
//    buffer_load ... lds pair (no VGPRs, out-of-range lanes read zero).
//  * The cells of the region are visited in 4 colour classes (cell parity in x and y).
//    Within a class no two cells share a node, so the element results go straight
//    into an LDS node accumulator with plain read-add-write (no two lanes or waves of
//    a class touch the same node); the classes are ordered
//    by barriers, so every node sums its (at most 4) cell contributions in a fixed
//    order: bitwise reproducible, no atomics to global memory, no gather pass.
//  * Uncut cells of a class: 16 per wave on the matrix cores, Y = K_ref [u_e1..u_e16]
//    (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64; K_ref fragments held in VGPRs).
//    Cut cells of a class add their products y_e = K_e u_e, computed once per step by
//    the cut-cell kernel (FP64 accumulation, rounded to the state precision).
//  * The update d_{k+1} = d_k + dt^2 M^{-1}(F_k - K u_k), u_{k+1} = u_k + d_{k+1} runs
//    row by row (lane = x); d and M^{-1} rows are staged in LDS at kernel entry.
#include <cstring>
#include <type_traits>

#include "step_common.h"

namespace fcw {

using Run2d = fcw_status (*)(hipStream_t, const void*, const int4*, int, int, const void*, int);

template <typename T>
__device__ static inline void buffer_dword_to_lds(__amdgpu_buffer_rsrc_t rsrc, int voffset,
                                                  void* lds_wave_base) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)lds_wave_base,
                                           4, voffset, 0, 0, 0);
}

// Per-problem arguments of a launch (device array, one entry per problem).
template <typename T>
struct Prob2d {
  T* ua;                 // caller state u (the final state of a call lands here)
  T* ub;                 // scratch (ping-pong partner of ua)
  T* d;                  // [nrhs][ndof]
  const T* invm;         // [nnodes]
  const int32_t* info;   // [ncells]
  const T* kref;         // [NL*NL]
  const T* ycut;         // [nrhs][ncand][NL] cut-cell products of this step
  int64_t ncand;
  const SourceDev* src;  // [nrhs] or null
  int n[2], np[2], ntile[2];
  int64_t ndof;
  double t0, dt;
  T dt2;
  int nsteps, start;
};

// SINGLE: one problem whose record comes by value; item = tile * nrhs + rhs.
template <typename T, int P, int TY, bool SINGLE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void step2d_kernel(
    const Prob2d<T>* __restrict__ probs, const int4* __restrict__ items, const Prob2d<T> one,
    int nrhs1, int nitems, int chunk, int j) {
  constexpr int NP1 = P + 1;
  constexpr int NL = NP1 * NP1;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  constexpr int TX = 64 / P;                 // one owned node row = one wave
  constexpr int OWX = TX * P;
  constexpr int RCX = TX + 1, RCY = TY + 1;  // region cells (tile + low ring)
  constexpr int NRC = RCX * RCY;
  constexpr int RNX = RCX * P + 1, RNY = RCY * P + 1;
  constexpr int W = RNX;                     // LDS row stride (elements)
  constexpr int DPE = sizeof(T) / 4;         // dwords per element
  constexpr int ROWDW = RNX * DPE;           // dwords per region row
  constexpr int NCH = (ROWDW + 63) / 64;     // 64-dword chunks per row
  constexpr int OWY = TY * P + 1;            // owned rows (at most)
  constexpr int NRW = (OWY + 3) / 4;         // owned rows per wave
  constexpr int NCI = (NRC + 255) / 256;
  static_assert(OWX <= 64, "tile row must fit one wave");
  static_assert(NMB * NKS <= 32, "K_ref fragments kept in registers");

  __shared__ T u_s[RNY * W];
  __shared__ T r_s[RNY * W];
  __shared__ T d_s[NRW * 4 * 64];    // owned rows of d, one wave-row each
  __shared__ T m_s[NRW * 4 * 64];    // owned rows of M^{-1}
  __shared__ int info_s[NRC];
  __shared__ double ft_s;
  __shared__ int src_on;

  // blocks b, b+8, ... run on one XCD: give them consecutive items
  const int item = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
  if (item >= nitems) return;
  const int4 wi = SINGLE ? make_int4(0, item % nrhs1, item / nrhs1, 0) : items[item];
  const Prob2d<T>& pr = SINGLE ? one : probs[wi.x];
  if (j >= pr.nsteps) return;  // this problem has finished its steps
  const int rhs = wi.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  const int tx = wi.z % pr.ntile[0], ty = wi.z / pr.ntile[0];
  const int cx0 = tx * TX, cy0 = ty * TY;
  const int rcx0 = cx0 - 1, rcy0 = cy0 - 1;
  const int rnx0 = rcx0 * P, rny0 = rcy0 * P;
  const int npx = pr.np[0], npy = pr.np[1];
  const int ox0 = cx0 * P, oy0 = cy0 * P;
  const int onx = (cx0 + TX >= pr.n[0]) ? npx - ox0 : OWX;  // OWX + 1 on the last full tile
  const int ony = (cy0 + TY >= pr.n[1]) ? npy - oy0 : TY * P;
  // ping-pong: the last step of a call writes ua
  const int par = (pr.nsteps - 1 - j) & 1;
  const int64_t roff = (int64_t)rhs * pr.ndof;
  const T* uin = (par ? pr.ua : pr.ub) + roff;
  T* dst_u = (par ? pr.ub : pr.ua) + roff;
  T* dst_d = pr.d + roff;
  const uint32_t nbytes = (uint32_t)((pr.n[0] * P + 1) * (int64_t)(pr.n[1] * P + 1) * sizeof(T));
  const __amdgpu_buffer_rsrc_t ursrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)uin, (short)0, (int)nbytes, 0x00020000);
  const double t = pr.t0 + j * pr.dt;

  // ---- entry: issue every load of the tile ----
  T areg[NMB][NKS];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int r = mb * 16 + lc, cc = 4 * kk + lk;
      const T v = pr.kref[min(r, NL - 1) * NL + min(cc, NL - 1)];
      areg[mb][kk] = (r < NL && cc < NL) ? v : T(0);
    }
  int inf_r[NCI];
#pragma unroll
  for (int it = 0; it < NCI; ++it) {
    const int c = tid + it * 256;
    const int gx = rcx0 + c % RCX, gy = rcy0 + c / RCX;
    const bool in = c < NRC && gx >= 0 && gx < pr.n[0] && gy >= 0 && gy < pr.n[1];
    const int v = pr.info[in ? gx + pr.n[0] * gy : 0];
    inf_r[it] = in ? v : kInfoOut;
  }
  // region rows straight into LDS; lanes left of the grid or past the array read 0,
  // lanes past a row end read the next row: both feed only cells outside the grid
  for (int ry = wave; ry < RNY; ry += 4) {
    const int gy = rny0 + ry;
    if (gy < 0 || gy >= npy) continue;
    const int rowbyte = (gy * npx + rnx0) * (int)sizeof(T);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int dw = ch * 64 + lane;
      if (ch < NCH - 1 || dw < ROWDW)
        buffer_dword_to_lds<T>(ursrc, rowbyte + dw * 4, (uint32_t*)(u_s + ry * W) + ch * 64);
    }
  }
  // owned rows of d and M^{-1}, straight into LDS as well (row oy -> slot oy)
  const __amdgpu_buffer_rsrc_t drsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_d, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t mrsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)pr.invm, (short)0, (int)nbytes, 0x00020000);
  for (int oy = wave; oy < ony; oy += 4) {
    const int rowbyte = ((oy0 + oy) * npx + ox0) * (int)sizeof(T);
#pragma unroll
    for (int ch = 0; ch < DPE; ++ch) {
      const int dw = ch * 64 + lane;
      buffer_dword_to_lds<T>(drsrc, rowbyte + dw * 4, (uint32_t*)(d_s + oy * 64) + ch * 64);
      buffer_dword_to_lds<T>(mrsrc, rowbyte + dw * 4, (uint32_t*)(m_s + oy * 64) + ch * 64);
    }
  }
  for (int i = tid; i < RNY * W; i += 256) r_s[i] = T(0);
#pragma unroll
  for (int it = 0; it < NCI; ++it) {
    const int c = tid + it * 256;
    if (c < NRC) info_s[c] = inf_r[it];
  }
  if (tid == 0) {
    src_on = 0;
    ft_s = 0.0;
    if (pr.src != nullptr) {
      const SourceDev& s = pr.src[rhs];
      const int sx0 = s.cell[0] * P, sy0 = s.cell[1] * P;
      if (sx0 + P >= ox0 && sx0 < ox0 + onx && sy0 + P >= oy0 && sy0 < oy0 + ony) {
        src_on = 1;
        ft_s = ricker(t, s.f0);
      }
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // ---- element products, colour class by colour class ----
  int offk[NKS];
#pragma unroll
  for (int kk = 0; kk < NKS; ++kk) {
    const int j = min(4 * kk + lk, NL - 1);
    offk[kk] = (j % NP1) + (j / NP1) * W;
  }
  // output rows of this lane (MFMA D layout) and their node offsets in a cell
  int offo[NMB][4];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = mb * 16 + Mma<T>::row(lk, r);
      offo[mb][r] = (i < NL) ? (i % NP1) + (i / NP1) * W : -1;
    }
  using Bits = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
#pragma unroll
  for (int color = 0; color < 4; ++color) {
    const int px = color & 1, py = color >> 1;
    const int nxc = (RCX - px + 1) / 2, nyc = (RCY - py + 1) / 2;
    const int ncol = nxc * nyc;
    // uncut cells of the class: 16 per wave on the matrix cores
    for (int b = wave; b * 16 < ncol; b += 4) {
      const int idx = min(b * 16 + lc, ncol - 1);
      const int lx = px + 2 * (idx % nxc), ly = py + 2 * (idx / nxc);
      const int c = lx + RCX * ly;
      const bool valid = (b * 16 + lc < ncol) && (info_s[c] == kInfoUncut);
      const int base = lx * P + ly * P * W;
      // every lane loads; invalid cells and padded rows are masked by bits (the
      // masked values may be stale LDS contents, never arithmetic on them)
      const Bits vmask = valid ? ~Bits(0) : Bits(0);
      T bv[NKS];
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk) {
        const Bits m = (4 * kk + lk < NL) ? vmask : Bits(0);
        const T v = u_s[base + offk[kk]];
        Bits vb;
        __builtin_memcpy(&vb, &v, sizeof(T));
        vb &= m;
        __builtin_memcpy(&bv[kk], &vb, sizeof(T));
      }
      typename Mma<T>::acc acc[NMB];
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) acc[mb] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[mb] = Mma<T>::mma(areg[mb][kk], bv[kk], acc[mb]);
      // read-add-write into the node accumulator: no two lanes or waves of a class
      // touch one node, so every node receives its contributions in class order; all
      // reads of the lane are issued before the first write
      T cur[NMB][4];
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) cur[mb][r] = r_s[base + max(offo[mb][r], 0)];
      if (valid) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (offo[mb][r] >= 0) r_s[base + offo[mb][r]] = cur[mb][r] + acc[mb][r];
      }
    }
    // cut cells of the class: their products come from the cut-cell kernel; one wave
    // per cell, lane = row
    int seen = 0;
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      const int idx = min(c0 + lane, ncol - 1);
      const int c = (px + 2 * (idx % nxc)) + RCX * (py + 2 * (idx / nxc));
      unsigned long long mask = __ballot(c0 + lane < ncol && info_s[c] >= 0);
      while (mask) {
        const int bit = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        if ((seen++ & 3) != wave) continue;
        const int ci = c0 + bit;
        const int lx = px + 2 * (ci % nxc), ly = py + 2 * (ci / nxc);
        const int q = info_s[lx + RCX * ly];
        const int base = lx * P + ly * P * W;
        const int i = min(lane, NL - 1);
        const T y = pr.ycut[((int64_t)rhs * pr.ncand + q) * NL + i];
        if (lane < NL) r_s[base + (i % NP1) + (i / NP1) * W] += y;
      }
    }
    __syncthreads();
  }

  // ---- update, one owned row per wave instruction ----
  const T dt2h = (pr.start && j == 0) ? T(0.5) * pr.dt2 : pr.dt2;
  const __amdgpu_buffer_rsrc_t drs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_d, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t urs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_u, (short)0, (int)nbytes, 0x00020000);
  const int nx64 = min(onx, OWX);
  const bool srcflag = src_on != 0;
  for (int oy = wave; oy < ony; oy += 4) {
    const int gy = oy0 + oy;
    const int rowbyte = (gy * npx + ox0) * (int)sizeof(T);
    const int rl0 = (ox0 - rnx0) + (gy - rny0) * W;
    if (lane < nx64) {
      const int rl = rl0 + lane;
      T F = T(0);
      if (srcflag) {
        const int sx = ox0 + lane - pr.src[rhs].cell[0] * P, sy = gy - pr.src[rhs].cell[1] * P;
        if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
      }
      const T dn = d_s[oy * 64 + lane] + dt2h * m_s[oy * 64 + lane] * (F - r_s[rl]);
      const T un = u_s[rl] + dn;
      const int vo = rowbyte + lane * (int)sizeof(T);
      if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, dn), drs, vo, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, un), urs, vo, 0, 0);
      } else {
        dst_d[(uint32_t)(gy * npx + ox0 + lane)] = dn;
        dst_u[(uint32_t)(gy * npx + ox0 + lane)] = un;
      }
    }
    if (onx > OWX && lane == 0) {  // the last node column of the grid
      const int gx = ox0 + OWX;
      const uint32_t node = (uint32_t)(gy * npx + gx);
      const int rl = rl0 + OWX;
      T F = T(0);
      if (srcflag) {
        const int sx = gx - pr.src[rhs].cell[0] * P, sy = gy - pr.src[rhs].cell[1] * P;
        if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
      }
      const T dn = dst_d[node] + dt2h * pr.invm[node] * (F - r_s[rl]);
      dst_d[node] = dn;
      dst_u[node] = u_s[rl] + dn;
    }
  }
}

// probs/items: device work list; when `one` is given (a host record of a single
// problem with nrhs1 right-hand sides) it is passed by value instead.
template <typename T, int P, int TY>
static fcw_status run2d(hipStream_t stream, const void* probs, const int4* items, int nitems,
                        int j, const void* one, int nrhs1) {
  const int chunk = (nitems + 7) / 8;
  if (one) {
    Prob2d<T> rec;
    std::memcpy(&rec, one, sizeof rec);
    step2d_kernel<T, P, TY, true><<<8 * chunk, 256, 0, stream>>>(nullptr, nullptr, rec, nrhs1,
                                                                 nitems, chunk, j);
  } else {
    step2d_kernel<T, P, TY, false><<<8 * chunk, 256, 0, stream>>>(
        (const Prob2d<T>*)probs, items, Prob2d<T>{}, 1, nitems, chunk, j);
  }
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

// 2-D step kernels offered to the autotuner: (P, TY) -> launcher; TX = 64 / P.
int step2d_candidates(int p, int fp64, int i, Run2d* fn, int tile[3]) {
  struct E { int p, ty; Run2d f32, f64; };
#define FCW_E(PP, TY) E{PP, TY, &run2d<float, PP, TY>, &run2d<double, PP, TY>}
  static const E table[] = {
      FCW_E(1, 16), FCW_E(1, 32), FCW_E(2, 8), FCW_E(2, 16), FCW_E(3, 8), FCW_E(3, 16),
      FCW_E(4, 8), FCW_E(4, 4), FCW_E(4, 16), FCW_E(5, 4), FCW_E(5, 8)};
#undef FCW_E
  int n = 0;
  for (const E& e : table) {
    if (e.p != p) continue;
    if (n == i) {
      if (fn) *fn = fp64 ? e.f64 : e.f32;
      if (tile) { tile[0] = 64 / e.p; tile[1] = e.ty; tile[2] = 1; }
    }
    ++n;
  }
  return n;
}

size_t prob2d_size(int fp64) { return fp64 ? sizeof(Prob2d<double>) : sizeof(Prob2d<float>); }

template <typename T>
static void fill_prob(const Ctx& c, void* out, void* ua, void* ub, void* d, double t0, double dt,
                      int nsteps, int start, int tx, int ty, const SourceDev* src) {
  Prob2d<T> p{};
  p.ua = (T*)ua;
  p.ub = (T*)ub;
  p.d = (T*)d;
  p.invm = (const T*)c.d_invm;
  p.info = c.d_info;
  p.kref = (const T*)c.d_kref_s;
  p.ycut = (const T*)c.d_ycut;
  p.ncand = c.n_cut_cand;
  p.src = src;
  p.n[0] = c.ncells[0];
  p.n[1] = c.ncells[1];
  p.np[0] = c.npts[0];
  p.np[1] = c.npts[1];
  p.ntile[0] = (c.ncells[0] + tx - 1) / tx;
  p.ntile[1] = (c.ncells[1] + ty - 1) / ty;
  p.ndof = c.ndof;
  p.t0 = t0;
  p.dt = dt;
  p.dt2 = (T)(dt * dt);
  p.nsteps = nsteps;
  p.start = start;
  std::memcpy(out, &p, sizeof p);
}

void prob2d_fill(const Ctx& c, void* out, void* ua, void* ub, void* d, double t0, double dt,
                 int nsteps, int start, int tx, int ty, const SourceDev* src) {
  if (c.precision == FCW_FP64)
    fill_prob<double>(c, out, ua, ub, d, t0, dt, nsteps, start, tx, ty, src);
  else
    fill_prob<float>(c, out, ua, ub, d, t0, dt, nsteps, start, tx, ty, src);
}

}  // namespace fcw
