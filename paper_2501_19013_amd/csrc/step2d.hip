// Central-difference step (paper eq. cdm) for 2-D scalar problems, shaped for CDNA4 wave64.
// One launch advances every item of a work list -- (problem, right-hand side, tile) --
// by one step, so several problems of one kind (same p and precision; any size,
// geometry and sources) and many right-hand sides share a launch.
//
//  * A tile is TX = 64 / P cells wide, so one owned node row of a tile is exactly one
//    wave (lane = x); TY cells high.  A workgroup (4 waves) stages the node values of
//    the tile plus one ring of cells on the low side in LDS, one region row per
//    buffer_load ... lds pair (no VGPRs, out-of-range lanes read zero).
//  * Element products of every cell of the region land in LDS (y_e per cell): uncut
//    cells 16 per wave on the matrix cores, Y = K_ref [u_e1..u_e16]
//    (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64; K_ref fragments held in VGPRs);
//    cut cells copy their products y_e = K_e u_e, computed once per step by the cut-cell
//    kernel (FP64 accumulation, rounded to the state precision).
//  * The update runs one owned node row per wave instruction (lane = x): each node
//    gathers its (at most 4) cell products in a fixed order -- lower cell row first,
//    lower cell first within a row -- so the sum is atomic-free and bitwise
//    reproducible; then d_{k+1} = d_k + dt^2 M^{-1}(F_k - K u_k), u_{k+1} = u_k + d_{k+1}.
//  * M^{-1} of a node whose cells are all uncut is the analytic product of 1-D inverse
//    GLL weights; only nodes flagged in a per-node bitmap (next to cut or outside cells)
//    read the stored inverse mass.  d and M^{-1} are loaded into registers during the
//    matrix-core phase.
#include <cstdio>
#include <cstring>
#include <string>
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

// s_waitcnt vmcnt(N) for a compile-time N (gfx9 encoding: vmcnt in bits 3:0 and 15:14;
// expcnt and lgkmcnt at their maxima, i.e. not waited for); a compiler barrier on both sides
template <int N>
__device__ static inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
  constexpr int imm = (N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(imm);
  asm volatile("" ::: "memory");
}

// One wave's 64 consecutive dwords, global -> LDS (lane l lands at lds_wave_base + 4 l).
__device__ static inline void lds_dword2d(const void* gsrc, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_wave_base, 4, 0,
                                   0);
}

// Per-problem arguments of a launch (device array, one entry per problem).
template <typename T>
struct Prob2d {
  T* ua;                 // caller state u (the final state of a call lands here)
  T* ub;                 // scratch (ping-pong partner of ua)
  T* d;                  // [nrhs][ndof]
  const T* invm;         // [nnodes], read where the node's flag bit is set
  const uint32_t* mflag; // [npy][wpr] per-node flag bits
  const double* invw;    // [npx + npy] 1-D inverse assembled GLL weights
  double cm;             // 1 / (rho (h/2)^2)
  int wpr;
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
__global__ __launch_bounds__(256) void step2d_kernel(
    const Prob2d<T>* __restrict__ probs, const int4* __restrict__ items, const Prob2d<T> one,
    int nrhs1, int nitems, int chunk, int j) {
  constexpr int NP1 = P + 1;
  constexpr int NL = NP1 * NP1;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  // y_s stride per cell: the padded MFMA rows plus 3, which spreads both the MFMA row
  // writes of 16 cells and the gather of a node row over the LDS banks
  constexpr int NLP = NMB * 16 + 3;
  constexpr int TX = 64 / P;                 // one owned node row = one wave
  constexpr int OWX = TX * P;
  constexpr int RCX = TX + 1, RCY = TY + 1;  // region cells (tile + low ring)
  constexpr int NRC = RCX * RCY;
  constexpr int NB = (NRC + 15) / 16;        // MFMA batches of 16 cells
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
  __shared__ T y_s[NRC * NLP];
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
  const uint32_t nbytes = (uint32_t)((int64_t)npx * npy * sizeof(T));
  const __amdgpu_buffer_rsrc_t ursrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)uin, (short)0, (int)nbytes, 0x00020000);
  const double t = pr.t0 + j * pr.dt;

  // ---- entry: every load of the tile is issued here and stays in flight ----
  // Nothing loaded is consumed before the single wait at the end of the entry: a use
  // would wait for every load issued before it (vmcnt counts in order).
  int inf_r[NCI];
#pragma unroll
  for (int it = 0; it < NCI; ++it) {
    const int c = tid + it * 256;
    const int gx = rcx0 + c % RCX, gy = rcy0 + c / RCX;
    const bool in = c < NRC && gx >= 0 && gx < pr.n[0] && gy >= 0 && gy < pr.n[1];
    inf_r[it] = pr.info[in ? gx + pr.n[0] * gy : 0];
  }
  int scell[2] = {-1 << 20, -1 << 20};
  double sf0 = 1.0;
  if (tid == 0 && pr.src != nullptr) {
    scell[0] = pr.src[rhs].cell[0];
    scell[1] = pr.src[rhs].cell[1];
    sf0 = pr.src[rhs].f0;
  }
  // flag words of the owned rows (uniform: scalar loads); the 64 nodes of a row from
  // ox0 on span at most three words
  uint32_t fw_r[NRW][3];
#pragma unroll
  for (int r = 0; r < NRW; ++r) {
    const int gy = min(oy0 + wave + 4 * r, npy - 1);
    const uint32_t* fw = pr.mflag + (size_t)gy * pr.wpr + (ox0 >> 5);
    fw_r[r][0] = fw[0];
    fw_r[r][1] = fw[1];
    fw_r[r][2] = fw[2];
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
  T areg[NMB][NKS];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int r = mb * 16 + lc, cc = 4 * kk + lk;
      areg[mb][kk] = pr.kref[min(r, NL - 1) * NL + min(cc, NL - 1)];
    }
  // d of the owned rows (lane = x) and the 1-D inverse weights of the analytic masses
  const int gx = ox0 + lane;
  const bool xin = lane < min(onx, OWX);
  const uint32_t node0 = (uint32_t)(oy0 * npx + gx);
  const double iwx = pr.invw[min(gx, npx - 1)];
  T d_r[NRW], im_r[NRW];
  double iwy_r[NRW];
#pragma unroll
  for (int r = 0; r < NRW; ++r) {
    const int oy = wave + 4 * r;
    // lanes and rows outside the owned box load node 0 (discarded): no branch, no
    // address outside the array
    const bool own = xin && oy < ony;
    const uint32_t node = own ? node0 + (uint32_t)(oy * npx) : 0u;
    const T dv = dst_d[node];
    d_r[r] = own ? dv : T(0);
    iwy_r[r] = pr.invw[npx + min(oy0 + oy, npy - 1)];
  }
  // stored inverse masses where the row's flag bit is set (the flags are scalar loads,
  // counted apart from the vector loads above)
  const int wsel = ((ox0 & 31) + lane) >> 5, wbit = (ox0 + lane) & 31;
  bool st_r[NRW];
#pragma unroll
  for (int r = 0; r < NRW; ++r) {
    const int oy = wave + 4 * r;
    const uint32_t word = (wsel == 0) ? fw_r[r][0] : (wsel == 1 ? fw_r[r][1] : fw_r[r][2]);
    st_r[r] = xin && oy < ony && ((word >> wbit) & 1u);
    im_r[r] = T(0);
    if (st_r[r]) im_r[r] = pr.invm[node0 + (uint32_t)(oy * npx)];
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
  for (int it = 0; it < NCI; ++it) {
    const int c = tid + it * 256;
    const int gx = rcx0 + c % RCX, gy = rcy0 + c / RCX;
    const bool in = c < NRC && gx >= 0 && gx < pr.n[0] && gy >= 0 && gy < pr.n[1];
    if (c < NRC) info_s[c] = in ? inf_r[it] : kInfoOut;
  }
  if (tid == 0) {
    const int sx0 = scell[0] * P, sy0 = scell[1] * P;
    const bool hit = pr.src != nullptr && sx0 + P >= ox0 && sx0 < ox0 + onx &&
                     sy0 + P >= oy0 && sy0 < oy0 + ony;
    src_on = hit ? 1 : 0;
    ft_s = hit ? ricker(t, sf0) : 0.0;
  }
  block_sync();

  // ---- element products of every region cell into y_s (stride NLP) ----
  {
    // B operand offsets of this lane's k rows; padded k rows read the cell's first node
    // (any finite value: the matching K_ref columns are zero)
    int offk[NKS];
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int jj = 4 * kk + lk;
      offk[kk] = (jj < NL) ? (jj % NP1) + (jj / NP1) * W : 0;
    }
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk)
        if (!(mb * 16 + lc < NL && 4 * kk + lk < NL)) areg[mb][kk] = T(0);
    // cut cells: their products (cut-cell kernel) go global -> LDS by DMA, one wave per
    // cell, all copies in flight while the matrix cores work below
    {
      int seen = 0;
      for (int c0 = 0; c0 < NRC; c0 += 64) {
        const int cq = c0 + lane;
        unsigned long long mask = __ballot(cq < NRC && info_s[min(cq, NRC - 1)] >= 0);
        while (mask) {
          const int bit = __ffsll((long long)mask) - 1;
          mask &= mask - 1;
          if ((seen++ & 3) != wave) continue;
          const int c = c0 + bit;
          const uint32_t* src =
              (const uint32_t*)(pr.ycut + ((int64_t)rhs * pr.ncand + info_s[c]) * NL);
          uint32_t* dst = (uint32_t*)(y_s + c * NLP);
#pragma unroll
          for (int ch = 0; ch < (NL * DPE + 63) / 64; ++ch)
            if (ch * 64 + lane < NL * DPE) lds_dword2d(src + ch * 64 + lane, dst + ch * 64);
        }
      }
    }
    // two batches of 16 cells per iteration: four independent accumulator chains
    for (int b0 = wave; b0 < NB; b0 += 8) {
      typename Mma<T>::acc acc[2][NMB];
      int cc[2], inf[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = (b0 + 4 * h) * 16 + lc;
        const int cs = min(c, NRC - 1);
        cc[h] = c;
        inf[h] = info_s[cs];
        const int base = (cs % RCX) * P + (cs / RCX) * P * W;
        T bv[NKS];
#pragma unroll
        for (int kk = 0; kk < NKS; ++kk) bv[kk] = u_s[base + offk[kk]];
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[h][mb] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NKS; ++kk)
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
            acc[h][mb] = Mma<T>::mma(areg[mb][kk], bv[kk], acc[h][mb]);
      }
      // uncut cells their product, outside cells zeros (a select: their operands may be
      // anything); cut cells were copied in above
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (cc[h] < NRC && inf[h] < 0) {
          const bool on = inf[h] == kInfoUncut;
          T* yo = y_s + cc[h] * NLP;
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              yo[mb * 16 + Mma<T>::row(lk, r)] = on ? acc[h][mb][r] : T(0);
        }
      }
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  block_sync();

  // ---- update, one owned row per wave instruction ----
  const T dt2h = (pr.start && j == 0) ? T(0.5) * pr.dt2 : pr.dt2;
  const __amdgpu_buffer_rsrc_t drs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_d, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t urs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_u, (short)0, (int)nbytes, 0x00020000);
  const bool srcflag = src_on != 0;
  // cells around node x = ox0 + lane (region-local): qx = lane / P + 1 with local lx, and
  // qx - 1 with local P when lx == 0 (lanes past the owned row, which store nothing,
  // are clamped into the region)
  const int qx = min(lane / P + 1, RCX - 1), lxl = lane % P;
  const T xam = (lxl == 0) ? T(1) : T(0);
  const int ymain = qx * NLP + lxl, ycorner = (qx - 1) * NLP + P;
  const int rxu = min(lane + P, RNX - 1);
#pragma unroll
  for (int r = 0; r < NRW; ++r) {
    const int oy = wave + 4 * r;
    if (oy >= ony) break;
    const int gy = oy0 + oy;
    const int ry = oy + P;  // region-local node row
    const int qy = ry / P, lyl = ry % P;
    // fixed order: the cell row below (when the node row is its top), then the row above
    // (when it exists); within a row the cell to the left first
    T acc = T(0);
    if (lyl == 0) {
      const T* yr = y_s + (qy - 1) * RCX * NLP + P * NP1;
      acc = acc + xam * yr[ycorner];
      acc = acc + yr[ymain];
    }
    if (gy < pr.n[1] * P) {
      const T* yr = y_s + qy * RCX * NLP + lyl * NP1;
      acc = acc + xam * yr[ycorner];
      acc = acc + yr[ymain];
    }
    if (xin) {
      T F = T(0);
      if (srcflag) {
        const int sx = gx - pr.src[rhs].cell[0] * P, sy = gy - pr.src[rhs].cell[1] * P;
        if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
      }
      const T im = st_r[r] ? im_r[r] : analytic_invm<T>(pr.cm, iwx, iwy_r[r], 1.0);
      const T dn = d_r[r] + dt2h * im * (F - acc);
      const T un = u_s[ry * W + rxu] + dn;
      const int vo = (gy * npx + gx) * (int)sizeof(T);
      if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, dn), drs, vo, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, un), urs, vo, 0, 0);
      } else {
        dst_d[(uint32_t)(gy * npx + gx)] = dn;
        dst_u[(uint32_t)(gy * npx + gx)] = un;
      }
    }
    if (onx > OWX && lane == 0) {  // the last node column of the grid (x = n_x P)
      const int gxe = ox0 + OWX;
      const uint32_t node = (uint32_t)(gy * npx + gxe);
      T acc2 = T(0);
      if (lyl == 0) acc2 = acc2 + y_s[((qy - 1) * RCX + RCX - 1) * NLP + P * NP1 + P];
      if (gy < pr.n[1] * P) acc2 = acc2 + y_s[(qy * RCX + RCX - 1) * NLP + lyl * NP1 + P];
      T F = T(0);
      if (srcflag) {
        const int sx = gxe - pr.src[rhs].cell[0] * P, sy = gy - pr.src[rhs].cell[1] * P;
        if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
      }
      const T dn = dst_d[node] + dt2h * pr.invm[node] * (F - acc2);
      dst_d[node] = dn;
      dst_u[node] = u_s[ry * W + OWX + P] + dn;
    }
  }
}

// Streaming variant: a block owns a column of TXS = 16 NBR - 1 cells (plus one ring cell
// on the left) and YR cell rows, and marches up the column one cell row at a time, so
// no cell row is computed twice and the loads of the next cell row are in flight while
// the current one is computed:
//  * node rows live in a ring buffer of 3P rows in LDS (row g in slot g mod 3P), filled
//    by buffer_load ... lds one cell row ahead; the cut-cell products of the next row go
//    global -> LDS the same way; d and the stored inverse masses of the next row's nodes
//    are loaded into registers one iteration ahead;
//  * per cell row, the NBR x NMB (16-cell batch, 16-row block) MFMA units are spread
//    over the waves; products land in one of three row buffers (previous, current,
//    next), so the node row shared with the previous cell row sums the previous row's
//    products first (the fixed order of the tile kernels);
//  * every store of the update is a buffer store with an out-of-range offset for lanes
//    that own no node, so each wave issues a fixed number of stores per row and the
//    end-of-row wait leaves exactly those in flight (vmcnt counts in issue order).
//  * PD = 2 (prefetch distance): the node rows, d and stored inverse masses of a cell row
//    are loaded two iterations ahead (ring of 4P rows), so their latency spans two
//    iterations; the cut-cell products stay one row ahead and are issued first, so the
//    end-of-row wait (a fixed count of later loads and stores per wave) covers them.
template <typename T, int P, int NBR, int YR, int NW, bool SINGLE, int PD>
__global__ __launch_bounds__(64 * NW, 24 / NW) void stream2d_kernel(
    const Prob2d<T>* __restrict__ probs, const int4* __restrict__ items, const Prob2d<T> one,
    int nrhs1, int nitems, int chunk, int j) {
  constexpr int NP1 = P + 1;
  constexpr int NL = NP1 * NP1;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  constexpr int NLP = NMB * 16 + 3;    // product stride per cell (bank-spread)
  constexpr int NCR = 16 * NBR;        // cells per row, ring cell included
  constexpr int TXS = NCR - 1;         // owned cells per row
  constexpr int RW = NCR * P + 1;      // node row width staged (from the ring cell)
  constexpr int OWN = TXS * P + 1;     // owned nodes per row at most (last column)
  constexpr int NH = (OWN + 63) / 64;  // wave-halves per node row
  constexpr int RING = (PD + 2) * P;   // ring buffer rows
  constexpr int DPE = sizeof(T) / 4;
  constexpr int RWD = RW * DPE;        // dwords per staged row
  constexpr int NCH = (RWD + 63) / 64;
  constexpr int NIR = YR + 1;          // cell rows with infos: cy0 - 1 .. cy0 + YR - 1
  constexpr int NNR = YR * P + 1;      // node rows of the block: cy0 P .. (cy0 + YR) P
  constexpr int FW = (OWN + 30) / 32 + 1;  // flag words spanned by a node row (any start)
  constexpr int NU = P * NH;           // update units (node row, half) per cell row
  constexpr int KU = (NU + NW - 1) / NW;  // units per wave
  constexpr int NMU = NBR * NMB;       // MFMA units per cell row
  static_assert(NMB * NKS <= 32, "K_ref fragments kept in registers");
  static_assert(PD == 1 || (PD == 2 && P % NW == 0),
                "prefetch distance 2 needs the same number of staged rows in every wave");
  // loads per wave that follow the cut-cell copies of a row (node rows, d, 1/M)
  constexpr int NFIX = NCH * (P / NW) + 2 * KU;

  __shared__ T u_r[RING * RW];
  __shared__ T y_b[3][NCR * NLP];
  __shared__ int info_s[NIR * NCR];
  __shared__ uint32_t fl_s[NNR * FW];
  __shared__ double iwy_s[NNR];
  __shared__ double ft_s;
  __shared__ int src_s[3];

  const int item = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
  if (item >= nitems) return;
  const int4 wi = SINGLE ? make_int4(0, item % nrhs1, item / nrhs1, 0) : items[item];
  const Prob2d<T>& pr = SINGLE ? one : probs[wi.x];
  if (j >= pr.nsteps) return;
  const int rhs = wi.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  const int cx0 = (wi.z % pr.ntile[0]) * TXS, cy0 = (wi.z / pr.ntile[0]) * YR;
  const int n0 = pr.n[0], n1 = pr.n[1];
  const int cy1 = min(cy0 + YR, n1);
  const int npx = pr.np[0], npy = pr.np[1];
  const int ox0 = cx0 * P, rnx0 = ox0 - P;
  const int onx = (cx0 + TXS >= n0) ? npx - ox0 : TXS * P;
  const int par = (pr.nsteps - 1 - j) & 1;
  const int64_t roff = (int64_t)rhs * pr.ndof;
  const T* uin = (par ? pr.ua : pr.ub) + roff;
  T* dst_u = (par ? pr.ub : pr.ua) + roff;
  T* dst_d = pr.d + roff;
  const uint32_t nbytes = (uint32_t)((int64_t)npx * npy * sizeof(T));
  const __amdgpu_buffer_rsrc_t urs_in =
      __builtin_amdgcn_make_buffer_rsrc((void*)uin, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t drs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_d, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t urs =
      __builtin_amdgcn_make_buffer_rsrc((void*)dst_u, (short)0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t mrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)pr.invm, (short)0, (int)nbytes, 0x00020000);
  constexpr uint32_t kOff = 0xFFFFFFF0u;  // out-of-range buffer offset: no access
  const double t = pr.t0 + j * pr.dt;

  // ring slot of node row g (g may be negative below the grid)
  auto slot = [](int g) { return ((g % RING) + RING) % RING; };
  // node rows [g0, g0 + nr) of u -> their ring slots (rows outside the grid read 0)
  auto stage_rows = [&](int g0, int nr) {
    for (int r = wave; r < nr; r += NW) {
      const int g = g0 + r;
      const uint32_t rowbyte = (uint32_t)(((int64_t)g * npx + rnx0) * (int)sizeof(T));
      T* dst = u_r + slot(g) * RW;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int dw = ch * 64 + lane;
        const uint32_t vo = (g >= 0 && g < npy) ? rowbyte + (uint32_t)dw * 4u : kOff;
        if (ch < NCH - 1 || dw < RWD)
          buffer_dword_to_lds<T>(urs_in, (int)vo, (uint32_t*)dst + ch * 64);
      }
    }
  };
  // cut-cell products of cell row cy into a row buffer, one wave per cell
  auto stage_cut = [&](int cy, T* yb) {
    const int* inf = info_s + (cy - (cy0 - 1)) * NCR;
    int seen = 0;
#pragma unroll
    for (int c0 = 0; c0 < NCR; c0 += 64) {
      const int cq = c0 + lane;
      unsigned long long mask = __ballot(cq < NCR && inf[min(cq, NCR - 1)] >= 0);
      while (mask) {
        const int bit = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        if ((seen++ % NW) != wave) continue;
        const int c = c0 + bit;
        const uint32_t* src =
            (const uint32_t*)(pr.ycut + ((int64_t)rhs * pr.ncand + inf[c]) * NL);
        uint32_t* dst = (uint32_t*)(yb + c * NLP);
#pragma unroll
        for (int ch = 0; ch < (NL * DPE + 63) / 64; ++ch)
          if (ch * 64 + lane < NL * DPE) lds_dword2d(src + ch * 64 + lane, dst + ch * 64);
      }
    }
  };

  // ---- prologue: the ring cell row's node rows (and, PD = 2, the first owned cell
  // row's) go first, so their loads overlap those of the infos, flags, 1-D inverse
  // weights and K_ref ----
  stage_rows((cy0 - 1) * P, P + 1);
  if constexpr (PD == 2) stage_rows(cy0 * P + 1, P);
  for (int i = tid; i < NIR * NCR; i += 64 * NW) {
    const int cy = cy0 - 1 + i / NCR, cx = cx0 - 1 + i % NCR;
    const bool in = cx >= 0 && cx < n0 && cy >= 0 && cy < n1;
    const int v = pr.info[in ? cx + n0 * cy : 0];
    info_s[i] = in ? v : kInfoOut;
  }
  for (int i = tid; i < NNR * FW; i += 64 * NW) {
    const int g = min(cy0 * P + i / FW, npy - 1);
    fl_s[i] = pr.mflag[(size_t)g * pr.wpr + (ox0 >> 5) + i % FW];
  }
  for (int i = tid; i < NNR; i += 64 * NW) iwy_s[i] = pr.invw[npx + min(cy0 * P + i, npy - 1)];
  if (tid == 0) {
    int sx = -(1 << 20), sy = -(1 << 20);
    double f = 0.0;
    if (pr.src != nullptr) {
      sx = pr.src[rhs].cell[0];
      sy = pr.src[rhs].cell[1];
      f = ricker(t, pr.src[rhs].f0);
    }
    src_s[0] = sx;
    src_s[1] = sy;
    src_s[2] = (sx * P + P >= ox0 && sx * P < ox0 + onx) ? 1 : 0;
    ft_s = f;
  }
  double iwx[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) iwx[h] = pr.invw[min(ox0 + h * 64 + lane, npx - 1)];
  T areg[NMB][NKS];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int r = mb * 16 + lc, cc = 4 * kk + lk;
      const T v = pr.kref[min(r, NL - 1) * NL + min(cc, NL - 1)];
      areg[mb][kk] = (r < NL && cc < NL) ? v : T(0);
    }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  block_sync();
  stage_cut(cy0 - 1, y_b[0]);

  // per-lane constants of the MFMA B operand: local node (ix, iy) of this lane's k rows
  int kx[NKS], ky[NKS];
#pragma unroll
  for (int kk = 0; kk < NKS; ++kk) {
    const int jj = 4 * kk + lk;
    kx[kk] = (jj < NL) ? jj % NP1 : 0;  // padded k rows read a real node (K_ref column 0)
    ky[kk] = (jj < NL) ? jj / NP1 : 0;
  }
  // update units of this wave: (node row in the cell row, half)
  T d_c[KU], d_n[KU], m_c[KU], m_n[KU], d_nn[KU], m_nn[KU];
  bool st_c[KU], st_n[KU], st_nn[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    d_n[k] = m_n[k] = d_nn[k] = m_nn[k] = T(0);
    st_n[k] = st_nn[k] = false;
  }
  // loads of the update operands of cell row cy (d; stored inverse masses where flagged)
  auto load_upd = [&](int cy, T* dr, T* mr, bool* sr) {
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      const int u = wave + NW * k;
      const int ly = u / NH, h = u % NH;
      const int g = cy * P + ly, xl = h * 64 + lane;
      const bool own = u < NU && xl < onx && g >= cy0 * P && g <= cy1 * P && g < npy;
      const uint32_t vo = own ? (uint32_t)(((int64_t)g * npx + ox0 + xl) * sizeof(T)) : kOff;
      const int fr = min(max(g - cy0 * P, 0), NNR - 1);
      const int gx = ox0 + xl;
      const uint32_t word = fl_s[fr * FW + min((gx >> 5) - (ox0 >> 5), FW - 1)];
      sr[k] = own && ((word >> (gx & 31)) & 1u);
      if constexpr (sizeof(T) == 4) {
        dr[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(drs, vo, 0, 0));
        mr[k] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(mrs, sr[k] ? vo : kOff, 0, 0));
      } else {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        dr[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(drs, vo, 0, 0));
        mr[k] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(mrs, sr[k] ? vo : kOff, 0, 0));
      }
    }
  };

  if constexpr (PD == 2) {
    // the first owned cell row's operands go ahead as well (its node rows came with the
    // ring row's)
    load_upd(cy0, d_nn, m_nn, st_nn);
  }
  const T dt2h = (pr.start && j == 0) ? T(0.5) * pr.dt2 : pr.dt2;
  int bp = 2, bc = 0, bn = 1;  // previous / current / next product buffers (distinct)
  for (int cy = cy0 - 1; cy < cy1; ++cy) {
    const bool ring = cy < cy0;
    // ---- A: loads of the next cell row(s) (all in flight during this row's work) ----
    if (cy + 1 < cy1) {
      stage_cut(cy + 1, y_b[bn]);
    }
    // nothing below moves above the cut-cell copies (the end-of-row wait counts on it)
    asm volatile("" ::: "memory");
    stage_rows((cy + PD) * P + 1, P);
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      d_c[k] = d_n[k];
      m_c[k] = m_n[k];
      st_c[k] = st_n[k];
      if constexpr (PD == 2) {
        d_n[k] = d_nn[k];
        m_n[k] = m_nn[k];
        st_n[k] = st_nn[k];
      }
    }
    if constexpr (PD == 2) load_upd(cy + 2, d_nn, m_nn, st_nn);
    else load_upd(cy + 1, d_n, m_n, st_n);

    // ---- B: products of cell row cy into y_b[bc] (cut cells were staged already) ----
    {
      const int* inf = info_s + (cy - (cy0 - 1)) * NCR;
      const int s0 = slot(cy * P);
      int offk[NKS];
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk) offk[kk] = ((s0 + ky[kk]) % RING) * RW + kx[kk];
      T* yb = y_b[bc];
      for (int un = wave; un < NMU; un += NW) {
        const int b = un / NMB, mb = un % NMB;
        const int c = b * 16 + lc;
        const int in = inf[c];
        T bv[NKS];
#pragma unroll
        for (int kk = 0; kk < NKS; ++kk) bv[kk] = u_r[offk[kk] + c * P];
        typename Mma<T>::acc acc = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NKS; ++kk) acc = Mma<T>::mma(areg[mb][kk], bv[kk], acc);
        if (in < 0) {
          const bool on = in == kInfoUncut;
#pragma unroll
          for (int r = 0; r < 4; ++r) yb[c * NLP + mb * 16 + Mma<T>::row(lk, r)] = on ? acc[r] : T(0);
        }
      }
    }
    block_sync();

    // ---- C: update of node rows cy P .. cy P + P - 1 ----
    if (!ring) {
      const T* yp = y_b[bp];
      const T* yc = y_b[bc];
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const int u = wave + NW * k;
        const int ly = min(u / NH, P - 1), h = u % NH;
        const int g = cy * P + ly, xl = h * 64 + lane;
        const bool own = u < NU && xl < onx;
        const int qx = min(xl / P + 1, NCR - 1), lx = xl % P;
        const T xam = (lx == 0) ? T(1) : T(0);
        T acc = T(0);
        if (ly == 0) {
          acc = acc + xam * yp[(qx - 1) * NLP + P * NP1 + P];
          acc = acc + yp[qx * NLP + P * NP1 + lx];
        }
        acc = acc + xam * yc[(qx - 1) * NLP + ly * NP1 + P];
        acc = acc + yc[qx * NLP + ly * NP1 + lx];
        T F = T(0);
        if (src_s[2]) {
          const int sx = ox0 + xl - src_s[0] * P, sy = g - src_s[1] * P;
          if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
        }
        const T im = st_c[k] ? m_c[k]
                             : analytic_invm<T>(pr.cm, iwx[min(h, NH - 1)],
                                                iwy_s[g - cy0 * P], 1.0);
        const T dn = d_c[k] + dt2h * im * (F - acc);
        const T un_ = u_r[slot(g) * RW + min(xl + P, RW - 1)] + dn;
        const uint32_t vo = own ? (uint32_t)(((int64_t)g * npx + ox0 + xl) * sizeof(T)) : kOff;
        if constexpr (sizeof(T) == 4) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, dn), drs, vo, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, un_), urs, vo, 0, 0);
        } else {
          typedef unsigned int u2 __attribute__((ext_vector_type(2)));
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, dn), drs, vo, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, un_), urs, vo, 0, 0);
        }
      }
      // PD = 1: the loads of the next row done; this row's 2 KU stores may still be in
      // flight.  PD = 2: besides, the NFIX loads of the row after next stay in flight.
      if constexpr (PD == 2) {
        wait_vmcnt<NFIX + 2 * KU>();
      } else {
        if constexpr (KU == 1) asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
        else if constexpr (KU == 2) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
        else if constexpr (KU == 3) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
        else if constexpr (KU == 4) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    block_sync();
    const int t3 = bp;
    bp = bc;
    bc = bn;
    bn = t3;
  }

  // ---- the top node row of the grid (only the cell row below contributes) ----
  static_assert(NH <= NW, "the top row takes one wave per half");
  if (cy1 == n1 && wave < NH) {
    const int g = n1 * P, h = wave, xl = h * 64 + lane;
    const bool own = xl < onx;
    const int qx = min(xl / P + 1, NCR - 1), lx = xl % P;
    const T xam = (lx == 0) ? T(1) : T(0);
    const T* yp = y_b[bp];
    T acc = T(0);
    acc = acc + xam * yp[(qx - 1) * NLP + P * NP1 + P];
    acc = acc + yp[qx * NLP + P * NP1 + lx];
    T F = T(0);
    if (src_s[2]) {
      const int sx = ox0 + xl - src_s[0] * P, sy = g - src_s[1] * P;
      if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * pr.src[rhs].b[sx + NP1 * sy]);
    }
    // unit (row 0, half h) of cell row n1 was loaded by wave h as its first unit
    const T im = st_n[0] ? m_n[0]
                         : analytic_invm<T>(pr.cm, iwx[min(h, NH - 1)], iwy_s[g - cy0 * P], 1.0);
    const T dn = d_n[0] + dt2h * im * (F - acc);
    const T un_ = u_r[slot(g) * RW + min(xl + P, RW - 1)] + dn;
    const uint32_t vo = own ? (uint32_t)(((int64_t)g * npx + ox0 + xl) * sizeof(T)) : kOff;
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, dn), drs, vo, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, un_), urs, vo, 0, 0);
    } else {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, dn), drs, vo, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, un_), urs, vo, 0, 0);
    }
  }
}

template <typename T, int P, int NBR, int YR, int NW, int PD>
static fcw_status runs2d(hipStream_t stream, const void* probs, const int4* items, int nitems,
                         int j, const void* one, int nrhs1) {
  const int chunk = (nitems + 7) / 8;
  if (one) {
    Prob2d<T> rec;
    std::memcpy(&rec, one, sizeof rec);
    stream2d_kernel<T, P, NBR, YR, NW, true, PD><<<8 * chunk, 64 * NW, 0, stream>>>(
        nullptr, nullptr, rec, nrhs1, nitems, chunk, j);
  } else {
    stream2d_kernel<T, P, NBR, YR, NW, false, PD><<<8 * chunk, 64 * NW, 0, stream>>>(
        (const Prob2d<T>*)probs, items, Prob2d<T>{}, 1, nitems, chunk, j);
  }
  FCW_HIP(hipGetLastError());
  return FCW_OK;
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

// 2-D step kernels offered to the autotuner: (P, TY) -> launcher; TX = 64 / P.  `name`
// receives the kernel's name as a profiler prints it (single-problem launches).
int step2d_candidates(int p, int fp64, int i, Run2d* fn, int tile[3], std::string* name) {
  struct E { int p, tx, ty, nbr, nw, pd; Run2d f32, f64; };
  // tile kernels (tile = cells), then streaming kernels (tile = owned cells per row x cell
  // rows per block)
#define FCW_S(PP, NBR, YR, NW) FCW_SD(PP, NBR, YR, NW, 1)
#define FCW_SD(PP, NBR, YR, NW, PD)                                  \
  E{PP, 16 * NBR - 1, YR, NBR, NW, PD, &runs2d<float, PP, NBR, YR, NW, PD>, \
    &runs2d<double, PP, NBR, YR, NW, PD>}
#define FCW_E(PP, TY) E{PP, 64 / PP, TY, 0, 0, 0, &run2d<float, PP, TY>, &run2d<double, PP, TY>}
  static const E table[] = {
      FCW_E(1, 4), FCW_E(1, 8), FCW_E(2, 8), FCW_E(2, 16), FCW_E(3, 8), FCW_E(3, 16),
      FCW_E(4, 8), FCW_E(4, 4), FCW_E(4, 16), FCW_E(5, 4), FCW_E(5, 8),
      FCW_S(2, 2, 8, 4), FCW_S(2, 2, 16, 4), FCW_S(3, 2, 8, 4), FCW_S(3, 2, 16, 4),
      FCW_S(4, 2, 3, 4), FCW_S(4, 2, 4, 4), FCW_S(4, 2, 5, 4), FCW_S(4, 2, 6, 4),
      FCW_S(4, 2, 8, 4), FCW_S(4, 2, 16, 4), FCW_S(4, 1, 4, 2), FCW_S(4, 1, 6, 2),
      FCW_S(4, 1, 8, 2), FCW_SD(4, 2, 4, 4, 2), FCW_SD(4, 2, 6, 4, 2), FCW_SD(4, 2, 8, 4, 2),
      FCW_SD(4, 2, 12, 4, 2), FCW_SD(4, 1, 6, 2, 2), FCW_SD(4, 1, 8, 2, 2)};
#undef FCW_E
#undef FCW_S
#undef FCW_SD
  int n = 0;
  for (const E& e : table) {
    if (e.p != p) continue;
    if (n == i) {
      if (fn) *fn = fp64 ? e.f64 : e.f32;
      if (tile) { tile[0] = e.tx; tile[1] = e.ty; tile[2] = 1; }
      if (name) {
        char b[128];
        const char* t = fp64 ? "double" : "float";
        if (e.nbr)
          std::snprintf(b, sizeof b, "fcw::stream2d_kernel<%s, %d, %d, %d, %d, true, %d>", t,
                        e.p, e.nbr, e.ty, e.nw, e.pd);
        else
          std::snprintf(b, sizeof b, "fcw::step2d_kernel<%s, %d, %d, true>", t, e.p, e.ty);
        *name = b;
      }
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
  p.mflag = c.d_mflag;
  p.invw = c.d_invw;
  p.cm = c.cm;
  p.wpr = c.mflag_wpr;
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
