// The explicit step of the spectral cell method on gfx950: one fused tile kernel per
// central-difference step (paper eq. cdm), organised for CDNA4:
//
//  * A workgroup (4 or 8 wave64) owns a tile of TX x TY (x TZ) cells and every node in the
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
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "step_common.h"
#include "zmarch.h"

namespace fcw {

// One wave's 64 consecutive dwords, global -> LDS without passing through registers
// (gfx950 global_load_lds_dword: lane l lands at lds_base + 4 l).
__device__ static inline void load_dword_to_lds(const void* gsrc, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_wave_base, 4, 0,
                                   0);
}

template <typename T, int DIM, int P, int NCOMP, int TX, int TY, int TZ, int MODE, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void tile_kernel(StepArgs<T> ain) {
  constexpr int NT = 64 * NW;  // threads of the block (NW waves)
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
  // bf16 operands (BF16 form): 16x16x32 MFMA, K_ref rows in k blocks of 32
  constexpr int NKB = (NL + 31) / 32;
  // split bf16 fragments of K_ref (hi, lo) in lane order: [mb][kb][hi/lo][lane] x 8 bf16
  constexpr int NFRAG = BF ? NMB * NKB * 2 * 64 : 1;
  constexpr int KWB = BF ? NKB * 32 : KW;
  constexpr bool AREG = !BF && NMB * NKS <= 32;  // keep K_ref fragments in VGPRs
  // otherwise stage them in LDS when small enough, else read them through the caches
  constexpr bool ALDS = !BF && !AREG && (NMB * 16 * KW * (int)sizeof(T) <= 48 * 1024);
  constexpr int NB = (NRC + 15) / 16;
  // owned node box of a tile (at most; edge tiles own one more node row)
  constexpr int OX = TX * P + 1;
  constexpr int OY = (DIM >= 2) ? TY * P + 1 : 1;
  constexpr int OZ = (DIM == 3) ? TZ * P + 1 : 1;
  constexpr int NO = (OX * OY * OZ + NT - 1) / NT;  // owned nodes per thread
  constexpr int NUV = NCOMP * NRN;                // staged node values
  constexpr int NUL = (NUV + NT - 1) / NT;            // ... per thread
  constexpr int NCI = (NRC + NT - 1) / NT;            // staged cell infos per thread
  // direct global->LDS staging of dword node values (the Lanczos operator scales them)
  constexpr bool DIRECT = (sizeof(T) == 4) && (MODE != kModeLanczos);

  // staged node values, plus one slot that holds zero: masked operands (padding of k,
  // cells other than uncut ones) read it, so every operand load is unconditional
  __shared__ T u_s[NUL * NT + 1];
  constexpr int ZSLOT = NUL * NT;
  __shared__ T y_s[NRC * NL];
  __shared__ T a_s[ALDS ? NMB * 16 * KW : 1];
  __shared__ int info_s[NRC];
  __shared__ int off_s[KWB];
  __shared__ bf16x8 a_sb[NFRAG];
  __shared__ double ft_s;
  __shared__ int src_on;

  // ---- the block's problem: the launch argument itself, or in a batched launch the
  // record of the problem whose block range holds this block ----
  StepArgs<T> a = ain;
  int bx = (int)blockIdx.x, nbk = (int)gridDim.x;
  if (MODE == kModeStep && ain.nprob > 0) {
    int pi = 0;
    while (pi + 1 < ain.nprob && ain.bstart[pi + 1] <= bx) ++pi;
    a = ain.probs[pi];
    const int j = ain.jstep;
    if (j >= a.nsteps || (int)blockIdx.y >= a.nrhs) return;
    bx -= ain.bstart[pi];
    nbk = ain.bstart[pi + 1] - ain.bstart[pi];
    // the state after step j of a call sits in the caller's buffer when nsteps - 1 - j is
    // even (the last step always writes it)
    T* ua = a.u_out;
    const bool par = ((a.nsteps - 1 - j) & 1) != 0;
    a.u_in = par ? ua : a.u_alt;
    a.u_out = par ? a.u_alt : ua;
    a.t = __dadd_rn(a.t0, __dmul_rn((double)j, a.dt));  // as the host forms t0 + j dt
    a.start = (a.start && j == 0) ? 1 : 0;
  }
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;

  // ---- once per block: K_ref fragments (registers or LDS) and the local offsets ----
  T areg[AREG ? NMB : 1][AREG ? NKS : 1];
  if (AREG) {
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk) {
        const int r = mb * 16 + lc, cc = 4 * kk + lk;
        const T* kp = (MODE == kModeLanczos) ? a.kref : a.kref;
        const T v = kp[min(r, NL - 1) * NL + min(cc, NL - 1)];
        areg[AREG ? mb : 0][AREG ? kk : 0] = (r < NL && cc < NL) ? v : T(0);
      }
  }
  if (ALDS) {
    for (int i = tid; i < NMB * 16 * KW; i += NT) {
      const int r = i / KW, cc = i % KW;
      a_s[i] = (r < NL && cc < NL) ? a.kref[r * NL + cc] : T(0);
    }
  }
  for (int j = tid; j < KWB; j += NT) {
    int off = -1;
    if (j < NL) {
      const int comp = j / NS, loc = j % NS;
      const int i0 = loc % NP1, i1 = (loc / NP1) % NP1, i2 = loc / (NP1 * NP1);
      off = comp * NRN + i0 + RNX * (i1 + RNY * i2);
    }
    off_s[j] = off;
  }
  if constexpr (BF) {
    // contiguous copy of the lane-ordered fragments (NFRAG x 16 bytes), 64 dwords per
    // wave instruction
    const uint32_t* src = (const uint32_t*)a.kref_bf;
    for (int w = wave; w < NFRAG * 4 / 64; w += NW)
      load_dword_to_lds(src + w * 64 + lane, (uint32_t*)a_sb + w * 64);
  }
  if (tid == 0) u_s[ZSLOT] = T(0);  // never written by the staging below
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  block_sync();

  // ---- the block's tiles: a stretch of the tiles of its XCD (blocks b, b + 8, ... run
  // on one XCD), so neighbouring tiles share halo rows in that XCD's L2 ----
  const int nbx = nbk / 8;
  // cell infos of the region of a tile (class or cut-cell index), one per thread and it
  auto load_info = [&](int tile, int out[NCI]) {
    const int rx = (tile % a.ntile[0]) * TX - 1;
    const int ry = (DIM >= 2) ? ((tile / a.ntile[0]) % a.ntile[1]) * TY - 1 : 0;
    const int rz = (DIM == 3) ? (tile / (a.ntile[0] * a.ntile[1])) * TZ - 1 : 0;
  #pragma unroll
    for (int it = 0; it < NCI; ++it) {
      const int c = tid + it * NT;
      const int gx = rx + c % RCX, gy = ry + (c / RCX) % RCY, gz = rz + c / (RCX * RCY);
      const bool in = c < NRC && gx >= 0 && gx < a.n[0] && gy >= 0 && gy < a.n[1] && gz >= 0 &&
                      gz < a.n[2];
      const int64_t cell = in ? gx + (int64_t)a.n[0] * (gy + (int64_t)a.n[1] * gz) : 0;
      const int v = a.info[cell];
      out[it] = in ? v : kInfoOut;
    }
  };
  // the next tile's infos are loaded one tile ahead, so its cut-cell copies can start
  // with its first loads
  int inf_next[NCI];
  {
    const int t0 = (bx % 8) * a.chunk + bx / 8;
    if (bx / 8 < a.chunk && t0 < a.ntiles) load_info(t0, inf_next);
  }
  for (int tk = bx / 8; tk < a.chunk; tk += nbx) {
    const int tile = (bx % 8) * a.chunk + tk;
    if (tile >= a.ntiles) break;
    const int tx = tile % a.ntile[0];
    const int ty = (DIM >= 2) ? (tile / a.ntile[0]) % a.ntile[1] : 0;
    const int tz = (DIM == 3) ? tile / (a.ntile[0] * a.ntile[1]) : 0;
    const int cx0 = tx * TX, cy0 = ty * TY, cz0 = tz * TZ;
    const int rcx0 = cx0 - 1;
    const int rcy0 = (DIM >= 2) ? cy0 - 1 : 0;
    const int rcz0 = (DIM == 3) ? cz0 - 1 : 0;
    const int rnx0 = rcx0 * P, rny0 = rcy0 * P, rnz0 = rcz0 * P;
    const T* uin = a.u_in + (int64_t)rhs * a.ndof;
    const int ox0 = cx0 * P;
    const int ox1 = (cx0 + TX >= a.n[0]) ? a.np[0] : (cx0 + TX) * P;
    const int oy0 = (DIM >= 2) ? cy0 * P : 0;
    const int oy1 = (DIM >= 2) ? ((cy0 + TY >= a.n[1]) ? a.np[1] : (cy0 + TY) * P) : 1;
    const int oz0 = (DIM == 3) ? cz0 * P : 0;
    const int oz1 = (DIM == 3) ? ((cz0 + TZ >= a.n[2]) ? a.np[2] : (cz0 + TZ) * P) : 1;
    const int onx = ox1 - ox0, ony = oy1 - oy0, onz = oz1 - oz0;

    // ---- issue every global load of the tile at once (all stay in flight) ----
    int inf_r[NCI];
  #pragma unroll
    for (int it = 0; it < NCI; ++it) inf_r[it] = inf_next[it];
    // cut cells: their products (cut-cell kernel) go global -> LDS by DMA first, each wave
    // copying the cut cells among its own lanes' cells
    if (MODE != kModeLanczos) {
      constexpr int DPE = (int)(sizeof(T) / 4);
      constexpr int RDW = NL * DPE;  // dwords of one cell's products
  #pragma unroll
      for (int it = 0; it < NCI; ++it) {
        unsigned long long mask = __ballot(inf_r[it] >= 0);
        while (mask) {
          const int bit = __ffsll((long long)mask) - 1;
          mask &= mask - 1;
          const int c = it * NT + wave * 64 + bit;
          const int q = __builtin_amdgcn_readlane(inf_r[it], bit);  // cut-cell index
          const uint32_t* src = (const uint32_t*)(a.ycut + ((int64_t)rhs * a.ncand + q) * NL);
          uint32_t* dst = (uint32_t*)(y_s + c * NL);
  #pragma unroll
          for (int ch = 0; ch < (RDW + 63) / 64; ++ch)
            if (ch * 64 + lane < RDW) load_dword_to_lds(src + ch * 64 + lane, dst + ch * 64);
        }
      }
    }
    // node values of the region; entries outside the grid belong only to cells outside
    // the grid (never read), so their address is clamped to node 0 of the component
    T u_r[DIRECT ? 1 : NUL];
  #pragma unroll
    for (int it = 0; it < NUL; ++it) {
      const int i = tid + it * NT;
      const int comp = min(i / NRN, NCOMP - 1), j = i % NRN;
      const int lx = j % RNX, ly = (j / RNX) % RNY, lz = j / (RNX * RNY);
      const int gx = rnx0 + lx, gy = rny0 + ly, gz = rnz0 + lz;
      const bool in = i < NUV && gx >= 0 && gx < a.np[0] && gy >= 0 && gy < a.np[1] && gz >= 0 &&
                      gz < a.np[2];
      const int64_t node = in ? gx + (int64_t)a.np[0] * (gy + (int64_t)a.np[1] * gz) : 0;
      const T* src = uin + (int64_t)comp * a.nnodes + node;
      if (DIRECT) {
        load_dword_to_lds(src, &u_s[it * NT + wave * 64]);
      } else {
        T v = *src;
        if (MODE == kModeLanczos) v = v * (T)sqrt(a.invm64[node]);
        u_r[DIRECT ? 0 : it] = in ? v : T(0);
      }
    }
    T d_r[MODE == kModeStep ? NO : 1][NCOMP];
    T im_r[MODE == kModeStep ? NO : 1];
    if (MODE == kModeStep) {
  #pragma unroll
      for (int it = 0; it < NO; ++it) {
        const int i = tid + it * NT;
        const int ii = (MODE == kModeStep) ? it : 0;
        const int lx = i % OX, ly = (i / OX) % OY, lz = i / (OX * OY);
        const bool own = i < OX * OY * OZ && lx < onx && ly < ony && lz < onz;
        const int64_t node =
            own ? (ox0 + lx) + (int64_t)a.np[0] * ((oy0 + ly) + (int64_t)a.np[1] * (oz0 + lz)) : 0;
        im_r[ii] = a.invm[node];
  #pragma unroll
        for (int comp = 0; comp < NCOMP; ++comp)
          d_r[ii][comp] = a.d[(int64_t)rhs * a.ndof + (int64_t)comp * a.nnodes + node];
      }
    }

    if (tk + nbx < a.chunk && tile + nbx < a.ntiles) load_info(tile + nbx, inf_next);

    // ---- stage cell info, node values, K_ref, local offsets in LDS ----
  #pragma unroll
    for (int it = 0; it < NCI; ++it) {
      const int c = tid + it * NT;
      if (c < NRC) info_s[c] = inf_r[it];
    }
    if (!DIRECT) {
  #pragma unroll
      for (int it = 0; it < NUL; ++it) u_s[tid + it * NT] = u_r[DIRECT ? 0 : it];
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
    if (DIRECT) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    block_sync();

    // ---- uncut cells: batched K_ref contraction on the matrix cores ----
    // Every non-cut cell of the region gets its row of y_s here: uncut cells their
    // product, cells outside the domain zeros (their B operand is masked to zero).
    if constexpr (BF) {
      // BF16 form: operands split into bf16 hi + lo parts (nearest even), the four products
      // K_lo u_lo + K_lo u_hi + K_hi u_lo + K_hi u_hi accumulated in FP32, smallest first
      for (int b = wave; b < NB; b += NW) {
        const int c = b * 16 + lc;
        const int cs = min(c, NRC - 1);
        const int inf = info_s[cs];
        const bool valid = (c < NRC) && (inf == kInfoUncut);
        if (__ballot(valid) == 0) {
          // no uncut cell among the 16: outside cells get their zero rows, no products
          if (c < NRC && inf == kInfoOut) {
  #pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
  #pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = mb * 16 + 4 * lk + r;
                if (i < NL) y_s[c * NL + i] = T(0);
              }
          }
          continue;
        }
        const int lx = cs % RCX, ly = (cs / RCX) % RCY, lz = cs / (RCX * RCY);
        const int base = lx * P + RNX * (ly * P + RNY * (lz * P));
        f32x4 acc[NMB];
  #pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[mb] = f32x4{0, 0, 0, 0};
        // every operand load of the block is issued before the first product
        float bv[NKB][8];
  #pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
  #pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int off = off_s[kb * 32 + 8 * lk + e];
            bv[kb][e] = (float)u_s[(valid && off >= 0) ? base + off : ZSLOT];
          }
        __builtin_amdgcn_sched_barrier(0);
  #pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
          bf16x8 bhi, blo;
  #pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)bv[kb][e];
            bhi[e] = h;
            blo[e] = (__bf16)(bv[kb][e] - (float)h);  // exact in FP32
          }
  #pragma unroll
          for (int mb = 0; mb < NMB; ++mb) {
            const bf16x8 ahi = a_sb[((mb * NKB + kb) * 2 + 0) * 64 + lane];
            const bf16x8 alo = a_sb[((mb * NKB + kb) * 2 + 1) * 64 + lane];
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, blo, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[mb], 0, 0, 0);
          }
        }
        if (c < NRC && inf < 0) {
  #pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
  #pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = mb * 16 + 4 * lk + r;
              if (i < NL) y_s[c * NL + i] = (T)acc[mb][r];
            }
        }
      }
    } else {
      int offk[NKS];
  #pragma unroll
      for (int kk = 0; kk < NKS; ++kk) offk[kk] = off_s[4 * kk + lk];
      for (int b = wave; b < NB; b += NW) {
        const int c = b * 16 + lc;
        const int cs = min(c, NRC - 1);
        const int inf = info_s[cs];
        const bool valid = (c < NRC) && (inf == kInfoUncut);
        if (__ballot(valid) == 0) {
          // no uncut cell among the 16: outside cells get their zero rows, no products
          if (c < NRC && inf == kInfoOut) {
  #pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
  #pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = mb * 16 + Mma<T>::row(lk, r);
                if (i < NL) y_s[c * NL + i] = T(0);
              }
          }
          continue;
        }
        const int lx = cs % RCX, ly = (cs / RCX) % RCY, lz = cs / (RCX * RCY);
        const int base = lx * P + RNX * (ly * P + RNY * (lz * P));
        T bv[NKS];
  #pragma unroll
        for (int kk = 0; kk < NKS; ++kk) {
          bv[kk] = u_s[(valid && offk[kk] >= 0) ? base + offk[kk] : ZSLOT];
        }
        // every operand load of the block is issued before the first product
        __builtin_amdgcn_sched_barrier(0);
        typename Mma<T>::acc acc[NMB];
  #pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[mb] = typename Mma<T>::acc{0, 0, 0, 0};
  #pragma unroll
        for (int kk = 0; kk < NKS; ++kk) {
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
            acc[mb] = Mma<T>::mma(av, bv[kk], acc[mb]);
          }
        }
        if (c < NRC && inf < 0) {
  #pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
  #pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = mb * 16 + Mma<T>::row(lk, r);
              if (i < NL) y_s[c * NL + i] = acc[mb][r];
            }
        }
      }
    }  // FP32 / FP64 operands

    // ---- Lanczos operator: full FP64 setup matrices streamed per tile, one wave per cell ----
    if (MODE == kModeLanczos) {
      int seen = 0;
      for (int c0 = 0; c0 < NRC; c0 += 64) {
        const int cc = c0 + lane;
        const bool isc = (cc < NRC) && (info_s[min(cc, NRC - 1)] >= 0);
        unsigned long long mask = __ballot(isc);
        while (mask) {
          const int bit = __ffsll((long long)mask) - 1;
          mask &= mask - 1;
          if ((seen++ % NW) != wave) continue;
          const int c = c0 + bit;
          const int q = info_s[c];
          const int lx = c % RCX, ly = (c / RCX) % RCY, lz = c / (RCX * RCY);
          const int base = lx * P + RNX * (ly * P + RNY * (lz * P));
          const T* K = a.kcut + (int64_t)q * NL * NL;
          constexpr int NR = (NL + 63) / 64;
          // FP64 accumulation: the rows of a cut-cell matrix cancel strongly and the
          // small lumped masses of cut-cell nodes amplify any error in their sum
          double y[NR];
  #pragma unroll
          for (int rr = 0; rr < NR; ++rr) y[rr] = 0.0;
          // straight-line over the columns: every load of the cell is issued before use
  #pragma unroll
          for (int j = 0; j < NL; ++j) {
            const T uj = u_s[base + off_s[j]];
  #pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
              const int i = min(lane + 64 * rr, NL - 1);
              y[rr] += (double)K[i * NL + j] * (double)uj;
            }
          }
  #pragma unroll
          for (int rr = 0; rr < NR; ++rr) {
            const int i = lane + 64 * rr;
            if (i < NL) y_s[c * NL + i] = (T)y[rr];
          }
        }
      }
    }
    if (MODE != kModeLanczos) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    block_sync();

    // ---- owned nodes: fixed-order gather of element results + update ----
    // The cells around node g along one axis are a = g/P - 1 (when g is a positive
    // multiple of P) and b = g/P (when g < n P); cells outside the domain hold zeros.
  #pragma unroll
    for (int it = 0; it < NO; ++it) {
      const int i = tid + it * NT;
      const int lx = i % OX, ly = (i / OX) % OY, lz = i / (OX * OY);
      if (i >= OX * OY * OZ || lx >= onx || ly >= ony || lz >= onz) continue;
      const int g3[3] = {ox0 + lx, oy0 + ly, oz0 + lz};
      const int64_t node = g3[0] + (int64_t)a.np[0] * (g3[1] + (int64_t)a.np[1] * g3[2]);
      int ca[3], cb[3], la[3], lb[3];
      bool ua[3], ub[3];
  #pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int rc0 = (k == 0) ? rcx0 : (k == 1 ? rcy0 : rcz0);
        if (k >= DIM) {
          ca[k] = cb[k] = 0; la[k] = lb[k] = 0; ua[k] = false; ub[k] = true;
          continue;
        }
        const int g = g3[k];
        const int q = g / P, rem = g - q * P;
        ua[k] = (rem == 0) && (g > 0);
        ub[k] = g < a.n[k] * P;
        ca[k] = max(q - 1 - rc0, 0);                       // region-local cell index
        cb[k] = min(q - rc0, (k == 0 ? RCX : (k == 1 ? RCY : RCZ)) - 1);
        la[k] = P;                                          // local node in cell a
        lb[k] = rem;                                        // local node in cell b
      }
      T r[NCOMP];
  #pragma unroll
      for (int comp = 0; comp < NCOMP; ++comp) r[comp] = T(0);
  #pragma unroll
      for (int sz = 0; sz < (DIM == 3 ? 2 : 1); ++sz)
  #pragma unroll
        for (int sy = 0; sy < (DIM >= 2 ? 2 : 1); ++sy)
  #pragma unroll
          for (int sx = 0; sx < 2; ++sx) {
            const bool use = (sx ? ub[0] : ua[0]) && (DIM < 2 || (sy ? ub[1] : ua[1])) &&
                             (DIM < 3 || (sz ? ub[2] : ua[2]));
            const int lcell = (sx ? cb[0] : ca[0]) +
                              RCX * ((sy ? cb[1] : ca[1]) + RCY * (sz ? cb[2] : ca[2]));
            const int loc = (sx ? lb[0] : la[0]) +
                            NP1 * ((sy ? lb[1] : la[1]) + NP1 * (sz ? lb[2] : la[2]));
  #pragma unroll
            for (int comp = 0; comp < NCOMP; ++comp) {
              const T v = y_s[lcell * NL + comp * NS + loc];
              r[comp] += use ? v : T(0);
            }
          }
      if (MODE == kModeStep) {
        const int ii = (MODE == kModeStep) ? it : 0;
        const int rl = (g3[0] - rnx0) + RNX * ((g3[1] - rny0) + RNY * (g3[2] - rnz0));
        const T im = im_r[ii];
        int sloc = -1;
        if (src_on) {
          const SourceDev& s = a.src[rhs];
          const int sx = g3[0] - s.cell[0] * P, sy = g3[1] - s.cell[1] * P,
                    sz = g3[2] - s.cell[2] * P;
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
          const T dn = d_r[ii][comp] + acc;
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
    block_sync();  // the next tile reuses the LDS
  }
}

// --------------------------------------------------------------------------------
// dispatch
// --------------------------------------------------------------------------------

// Blocks per XCD of a persistent launch: as many as the kernel's occupancy keeps resident
// on the XCD's compute units (at most one per tile).
static int resident_per_xcd(const void* kern, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kern);
  if (it != cache.end()) return it->second;
  int dev = 0, ncu = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, 0) != hipSuccess || nb < 1)
    return 64;  // a safe guess; not cached
  const int v = std::max(1, nb * ncu / 8);
  cache[kern] = v;
  return v;
}

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

using RunFn = fcw_status (*)(Ctx&, int, int, const void*, void*, void*, double, double, int);

// A step configuration's batched form (several problems of its kind per launch).
struct BatchOps {
  int (*blocks_per_xcd)();                  // resident blocks per XCD of the kernel
  int (*ntiles)(const Ctx&);                // tiles of a problem
  // record of one problem's call: caller state ua, partner ub, increment d, time origin,
  // step, step count, start flag, right-hand sides
  void (*fill)(Ctx&, void*, void*, void*, void*, double, double, int, int, int);
  fcw_status (*run)(hipStream_t, const void*, const int32_t*, int, int, int, int);
  size_t rec_size;
};

template <typename T, int DIM, int P, int NCOMP, int TX, int TY, int TZ, bool BF = false, int NW = 4>
struct TileCfg {
  // 3-D: persistent launch, 8 x (blocks per XCD) blocks each walking its XCD's tiles, so
  // the large K_ref (LDS or bf16 fragments) is staged once per block; 2-D (K_ref in
  // registers): one block per tile, which balances better
  static fcw_status launch(void (*kern)(StepArgs<T>), Ctx& c, const StepArgs<T>& a, int nrhs) {
    const int nbx =
        (DIM == 3) ? std::min(a.chunk, resident_per_xcd((const void*)kern, 64 * NW)) : a.chunk;
    kern<<<dim3(8 * nbx, nrhs, 1), 64 * NW, 0, c.stream>>>(a);
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
  static StepArgs<T> args(Ctx& c, const void* uin, void* uout, void* d, double t, double dt,
                          int start, int mode) {
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
    a.ycut = (const T*)c.d_ycut;
    a.ncand = c.n_cut_cand;
    a.kref_bf = c.d_kref_bf;
    return a;
  }
  // every mode (the default configuration of a problem kind)
  static fcw_status run(Ctx& c, int mode, int nrhs, const void* uin, void* uout, void* d,
                        double t, double dt, int start) {
    if (mode != kModeLanczos && !c.skip_cut) {
      fcw_status st = launch_cut_products(c, nrhs, uin);
      if (st) return st;
    }
    StepArgs<T> a = args(c, uin, uout, d, t, dt, start, mode);
    if (mode == kModeStep) return launch(tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeStep, BF, NW>, c, a, nrhs);
    if (mode == kModeApply)
      return launch(tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeApply, BF, NW>, c, a, nrhs);
    return launch(tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeLanczos, false, NW>, c, a, nrhs);
  }
  // the step only (alternative tile shapes offered to the autotuner)
  static fcw_status run_step(Ctx& c, int mode, int nrhs, const void* uin, void* uout, void* d,
                             double t, double dt, int start) {
    if (mode != kModeStep) {
      set_error("tile configuration built for the step only");
      return FCW_E_UNSUPPORTED;
    }
    if (!c.skip_cut) {
      fcw_status st = launch_cut_products(c, nrhs, uin);
      if (st) return st;
    }
    StepArgs<T> a = args(c, uin, uout, d, t, dt, start, mode);
    return launch(tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeStep, BF, NW>, c, a, nrhs);
  }
  // ---- batched form ----
  static int blocks_per_xcd() {
    return resident_per_xcd(
        (const void*)tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeStep, BF, NW>, 64 * NW);
  }
  static int ntiles(const Ctx& c) { return make_args<T>(c, TX, TY, TZ).ntiles; }
  static void fill(Ctx& c, void* out, void* ua, void* ub, void* d, double t0, double dt,
                   int nsteps, int start, int nrhs) {
    StepArgs<T> a = args(c, ua, ua, d, t0, dt, start, kModeStep);
    a.u_alt = (T*)ub;
    a.t0 = t0;
    a.dt = dt;
    a.nsteps = nsteps;
    a.nrhs = nrhs;
    std::memcpy(out, &a, sizeof a);
  }
  static fcw_status run_batch(hipStream_t s, const void* recs, const int32_t* bstart, int nprob,
                              int nblocks, int maxrhs, int j) {
    StepArgs<T> a{};
    a.probs = (const StepArgs<T>*)recs;
    a.bstart = bstart;
    a.nprob = nprob;
    a.jstep = j;
    tile_kernel<T, DIM, P, NCOMP, TX, TY, TZ, kModeStep, BF, NW>
        <<<dim3(nblocks, maxrhs, 1), 64 * NW, 0, s>>>(a);
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
  static const BatchOps* ops() {
    static const BatchOps o{&blocks_per_xcd, &ntiles, &fill, &run_batch, sizeof(StepArgs<T>)};
    return &o;
  }
};

// 3-D z-marching kernel (zmarch.h): tile = (TX, TY, cell layers per item); the state
// of one right-hand side must stay below 2 GiB (32-bit buffer offsets)
template <typename T, int P, int NCOMP, int TX, int TY, int ZR, int NW>
struct ZCfg {
  using Base = TileCfg<T, 3, P, NCOMP, TX, TY, ZR, false, NW>;
  static constexpr void (*kern)(StepArgs<T>) = zmarch_kernel<T, P, NCOMP, TX, TY, ZR, NW>;
  static bool fits(const Ctx& c) {
    return c.ndof * (int64_t)sizeof(T) < 0x7FFFFFF0 && c.ncells[0] * (int64_t)c.ncells[1] *
                                                               c.ncells[2] * 4 < 0x7FFFFFF0;
  }
  static fcw_status run_step(Ctx& c, int mode, int nrhs, const void* uin, void* uout, void* d,
                             double t, double dt, int start) {
    if (mode != kModeStep || !fits(c)) {
      set_error("z-marching kernel: step mode and states below 2 GiB only");
      return FCW_E_UNSUPPORTED;
    }
    if (!c.skip_cut) {
      fcw_status st = launch_cut_products(c, nrhs, uin);
      if (st) return st;
    }
    StepArgs<T> a = Base::args(c, uin, uout, d, t, dt, start, kModeStep);
    const int nbx = std::min(a.chunk, resident_per_xcd((const void*)kern, 64 * NW));
    kern<<<dim3(8 * nbx, nrhs, 1), 64 * NW, 0, c.stream>>>(a);
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
  static int blocks_per_xcd() { return resident_per_xcd((const void*)kern, 64 * NW); }
  static fcw_status run_batch(hipStream_t s, const void* recs, const int32_t* bstart, int nprob,
                              int nblocks, int maxrhs, int j) {
    StepArgs<T> a{};
    a.probs = (const StepArgs<T>*)recs;
    a.bstart = bstart;
    a.nprob = nprob;
    a.jstep = j;
    kern<<<dim3(nblocks, maxrhs, 1), 64 * NW, 0, s>>>(a);
    FCW_HIP(hipGetLastError());
    return FCW_OK;
  }
  static const BatchOps* ops() {
    static const BatchOps o{&blocks_per_xcd, &Base::ntiles, &Base::fill, &run_batch,
                            sizeof(StepArgs<T>)};
    return &o;
  }
};

struct Cand {
  RunFn fn;
  int tile[3];
  int nw;  // waves per block
  const BatchOps* ops;
  bool zm = false;  // the z-marching kernel
};

// Candidate tile shapes per problem kind; entry 0 is the default and serves every mode.
template <typename T>
static int candidates(const Ctx& c, Cand* out) {
  constexpr bool F64 = sizeof(T) == 8;
  int n = 0;
#define FCW_C0(D, PP, NC, TX, TY, TZ)                  \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<T, D, PP, NC, TX, TY, TZ>::run, {TX, TY, TZ}, 4,              \
                    TileCfg<T, D, PP, NC, TX, TY, TZ>::ops()};
#define FCW_C(D, PP, NC, TX, TY, TZ)                   \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<T, D, PP, NC, TX, TY, TZ>::run_step, {TX, TY, TZ}, 4,         \
                    TileCfg<T, D, PP, NC, TX, TY, TZ>::ops()};
#define FCW_CW(D, PP, NC, TX, TY, TZ, NW)              \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<T, D, PP, NC, TX, TY, TZ, false, NW>::run_step, {TX, TY, TZ}, NW, \
                    TileCfg<T, D, PP, NC, TX, TY, TZ, false, NW>::ops()};
#define FCW_CZ(PP, NC, TX, TY, ZR, NW)                 \
  if (c.dim == 3 && c.p == PP && c.ncomp == NC && ZCfg<T, PP, NC, TX, TY, ZR, NW>::fits(c)) \
    out[n++] = Cand{&ZCfg<T, PP, NC, TX, TY, ZR, NW>::run_step, {TX, TY, ZR}, NW,           \
                    ZCfg<T, PP, NC, TX, TY, ZR, NW>::ops(), true};
  if constexpr (F64) {
    FCW_C0(2, 1, 1, 32, 16, 1) FCW_C(2, 1, 1, 16, 16, 1)
    FCW_C0(2, 2, 1, 16, 16, 1) FCW_C(2, 2, 1, 16, 8, 1)
    FCW_C0(2, 3, 1, 16, 8, 1) FCW_C(2, 3, 1, 8, 8, 1)
    FCW_C0(2, 4, 1, 16, 8, 1) FCW_C(2, 4, 1, 8, 8, 1) FCW_C(2, 4, 1, 8, 4, 1)
    FCW_C0(2, 5, 1, 8, 8, 1) FCW_C(2, 5, 1, 8, 4, 1)
    FCW_C0(2, 6, 1, 8, 8, 1) FCW_C(2, 6, 1, 8, 4, 1)
    FCW_C0(3, 1, 1, 8, 8, 4)
    FCW_C0(3, 2, 1, 8, 4, 4) FCW_C(3, 2, 1, 4, 4, 4)
    FCW_C0(3, 3, 1, 4, 4, 4) FCW_C(3, 3, 1, 4, 4, 2)
    FCW_C0(3, 4, 1, 4, 4, 2) FCW_C(3, 4, 1, 4, 2, 2)
    FCW_C0(3, 1, 3, 8, 4, 4)
    FCW_C0(3, 2, 3, 4, 4, 2) FCW_C(3, 2, 3, 4, 2, 2)
    FCW_C0(3, 3, 3, 4, 2, 2)
  } else {
    FCW_C0(2, 1, 1, 32, 32, 1) FCW_C(2, 1, 1, 32, 16, 1)
    FCW_C0(2, 2, 1, 16, 16, 1) FCW_C(2, 2, 1, 16, 8, 1) FCW_C(2, 2, 1, 32, 16, 1)
    FCW_C0(2, 3, 1, 16, 16, 1) FCW_C(2, 3, 1, 16, 8, 1) FCW_C(2, 3, 1, 8, 8, 1)
    FCW_C0(2, 4, 1, 16, 16, 1) FCW_C(2, 4, 1, 16, 8, 1) FCW_C(2, 4, 1, 8, 8, 1)
    FCW_C(2, 4, 1, 32, 8, 1) FCW_C(2, 4, 1, 8, 4, 1)
    FCW_C0(2, 5, 1, 16, 8, 1) FCW_C(2, 5, 1, 8, 8, 1)
    FCW_C0(2, 6, 1, 8, 8, 1) FCW_C(2, 6, 1, 8, 4, 1)
    FCW_C0(3, 1, 1, 8, 8, 8)
    FCW_C0(3, 2, 1, 8, 4, 4) FCW_C(3, 2, 1, 4, 4, 4) FCW_C(3, 2, 1, 8, 8, 4)
    FCW_C0(3, 3, 1, 4, 4, 4) FCW_C(3, 3, 1, 4, 4, 2)
    FCW_C0(3, 4, 1, 4, 4, 2) FCW_C(3, 4, 1, 4, 2, 2)
    FCW_C0(3, 1, 3, 8, 4, 4)
    FCW_C0(3, 2, 3, 4, 4, 4) FCW_C(3, 2, 3, 4, 4, 2) FCW_C(3, 2, 3, 4, 2, 2)
    FCW_CW(3, 2, 3, 4, 4, 4, 8) FCW_CW(3, 2, 3, 8, 4, 4, 8)
    FCW_C0(3, 3, 3, 4, 2, 2) FCW_C(3, 3, 3, 4, 4, 2)
    FCW_CW(3, 3, 3, 4, 2, 2, 8) FCW_CW(3, 3, 3, 4, 4, 2, 8) FCW_CW(3, 3, 3, 4, 4, 4, 8)
    FCW_CW(3, 3, 3, 8, 4, 2, 8)
    FCW_CZ(2, 3, 8, 8, 16, 6) FCW_CZ(2, 3, 8, 8, 32, 6)
    FCW_CZ(2, 3, 8, 4, 16, 6) FCW_CZ(2, 3, 8, 4, 32, 6)
  }
#undef FCW_C0
#undef FCW_C
#undef FCW_CW
#undef FCW_CZ
  return n;
}

constexpr int kMaxCand = 16;

// BF16 form: FP32 state, bf16 operands of the uncut contraction
static int candidates_bf(const Ctx& c, Cand* out) {
  int n = 0;
#define FCW_B0(D, PP, NC, TX, TY, TZ)                  \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<float, D, PP, NC, TX, TY, TZ, true>::run, {TX, TY, TZ}, 4,    \
                    TileCfg<float, D, PP, NC, TX, TY, TZ, true>::ops()};
#define FCW_B(D, PP, NC, TX, TY, TZ)                   \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<float, D, PP, NC, TX, TY, TZ, true>::run_step, {TX, TY, TZ}, 4, \
                    TileCfg<float, D, PP, NC, TX, TY, TZ, true>::ops()};
#define FCW_BW(D, PP, NC, TX, TY, TZ, NW)              \
  if (c.dim == D && c.p == PP && c.ncomp == NC)        \
    out[n++] = Cand{&TileCfg<float, D, PP, NC, TX, TY, TZ, true, NW>::run_step, {TX, TY, TZ}, \
                    NW, TileCfg<float, D, PP, NC, TX, TY, TZ, true, NW>::ops()};
  FCW_B0(2, 1, 1, 32, 32, 1)
  FCW_B0(2, 2, 1, 16, 16, 1) FCW_B(2, 2, 1, 16, 8, 1)
  FCW_B0(2, 3, 1, 16, 16, 1) FCW_B(2, 3, 1, 16, 8, 1)
  FCW_B0(2, 4, 1, 16, 8, 1) FCW_B(2, 4, 1, 16, 16, 1) FCW_B(2, 4, 1, 8, 8, 1)
  FCW_B0(2, 5, 1, 16, 8, 1) FCW_B(2, 5, 1, 8, 8, 1)
  FCW_B0(2, 6, 1, 8, 8, 1)
  FCW_B0(3, 1, 1, 8, 8, 8)
  FCW_B0(3, 2, 1, 8, 4, 4) FCW_B(3, 2, 1, 4, 4, 4)
  FCW_B0(3, 3, 1, 4, 4, 4) FCW_B(3, 3, 1, 4, 4, 2)
  FCW_B0(3, 4, 1, 4, 4, 2) FCW_B(3, 4, 1, 4, 2, 2)
  FCW_B0(3, 1, 3, 8, 4, 4)
  FCW_B0(3, 2, 3, 4, 4, 2) FCW_B(3, 2, 3, 4, 4, 4) FCW_B(3, 2, 3, 4, 2, 2)
  FCW_BW(3, 2, 3, 4, 4, 4, 8) FCW_BW(3, 2, 3, 8, 4, 4, 8)
#undef FCW_B0
#undef FCW_B
#undef FCW_BW
  return n;
}

static int cands_for(const Ctx& c, bool fp64, Cand* out) {
  if (!fp64 && c.precision == FCW_BF16) return candidates_bf(c, out);
  return fp64 ? candidates<double>(c, out) : candidates<float>(c, out);
}

static RunFn select_for(const Ctx& c, bool fp64, int choice = 0) {
  Cand cs[kMaxCand];
  const int n = cands_for(c, fp64, cs);
  if (n == 0) return nullptr;
  if (choice < 0 || choice >= n) choice = 0;
  return cs[choice].fn;
}

bool step_supported(const Ctx& c) {
  return select_for(c, c.precision == FCW_FP64) != nullptr && select_for(c, true) != nullptr;
}

using Run2d = fcw_status (*)(hipStream_t, const void*, const int4*, int, int, const void*, int);
int step2d_candidates(int p, int fp64, int i, Run2d* fn, int tile[3], std::string* name);
size_t prob2d_size(int fp64);
void prob2d_fill(const Ctx& c, void* out, void* ua, void* ub, void* d, double t0, double dt,
                 int nsteps, int start, int tx, int ty, const SourceDev* src);

// Step configurations offered to the autotuner: the work-list 2-D kernels (step2d.hip)
// for 2-D scalar problems, then the tile shapes of the generic kernel.
struct StepCand {
  Run2d f2d = nullptr;
  RunFn fgen = nullptr;
  int tile[3] = {0, 0, 0};
  int nw = 4;
  bool zm = false;
};

static int step_candidates(const Ctx& c, int i, StepCand* out) {
  const int fp64 = c.precision == FCW_FP64;
  const int n2 = (c.dim == 2 && c.ncomp == 1 && c.precision != FCW_BF16)
                     ? step2d_candidates(c.p, fp64, -1, nullptr, nullptr, nullptr)
                     : 0;
  Cand cs[kMaxCand];
  const int ng = cands_for(c, fp64, cs);
  if (out) {
    if (i >= 0 && i < n2) {
      step2d_candidates(c.p, fp64, i, &out->f2d, out->tile, nullptr);
    } else if (i >= n2 && i < n2 + ng) {
      out->fgen = cs[i - n2].fn;
      for (int k = 0; k < 3; ++k) out->tile[k] = cs[i - n2].tile[k];
      out->nw = cs[i - n2].nw;
      out->zm = cs[i - n2].zm;
    }
  }
  return n2 + ng;
}

int tile_candidates(const Ctx& c, int i, int tile[3], std::string* name) {
  StepCand sc;
  const int n = step_candidates(c, i, &sc);
  if (i < 0 || i >= n) return n;
  if (tile)
    for (int k = 0; k < 3; ++k) tile[k] = sc.tile[k];
  if (name && sc.f2d) {
    step2d_candidates(c.p, c.precision == FCW_FP64, i, nullptr, nullptr, name);
  } else if (name && sc.zm) {
    char b[128];
    std::snprintf(b, sizeof b, "fcw::zmarch_kernel<%s, %d, %d, %d, %d, %d, %d>",
                  c.precision == FCW_FP64 ? "double" : "float", c.p, c.ncomp, sc.tile[0],
                  sc.tile[1], sc.tile[2], sc.nw);
    *name = b;
  } else if (name) {
    // the kernel's name as a profiler prints it (single-problem launches)
    char b[128];
    std::snprintf(b, sizeof b, "fcw::tile_kernel<%s, %d, %d, %d, %d, %d, %d, %d, %s, %d>",
                  c.precision == FCW_FP64 ? "double" : "float", c.dim, c.p, c.ncomp, sc.tile[0],
                  sc.tile[1], sc.tile[2], (int)kModeStep,
                  c.precision == FCW_BF16 ? "true" : "false", sc.nw);
    *name = b;
  }
  return n;
}

// Device work list (problem records + items) with pinned staging, owned by `c`.
static fcw_status stage_worklist(Ctx& c, const void* host, size_t bytes) {
  if (c.wl_bytes < bytes) {
    if (c.wl_event) FCW_HIP(hipEventSynchronize(c.wl_event));
    if (c.d_wl) FCW_HIP(hipFree(c.d_wl));
    if (c.h_wl) FCW_HIP(hipHostFree(c.h_wl));
    c.d_wl = nullptr;
    c.h_wl = nullptr;
    FCW_HIP(hipMalloc(&c.d_wl, bytes));
    FCW_HIP(hipHostMalloc(&c.h_wl, bytes, hipHostMallocDefault));
    c.wl_bytes = bytes;
  }
  // the pinned staging buffer may still feed a previous copy
  if (c.wl_event) FCW_HIP(hipEventSynchronize(c.wl_event));
  else FCW_HIP(hipEventCreateWithFlags(&c.wl_event, hipEventDisableTiming));
  std::memcpy(c.h_wl, host, bytes);
  FCW_HIP(hipMemcpyAsync(c.d_wl, c.h_wl, bytes, hipMemcpyHostToDevice, c.stream));
  FCW_HIP(hipEventRecord(c.wl_event, c.stream));
  return FCW_OK;
}

// The launches of one step of a batched group: the cut-cell products of every member
// that has cut cells, then the 2-D kernel over all items.
static fcw_status group_step(Ctx& owner, Run2d fn, const void* dprobs, const int4* ditems,
                             int nitems, const void* dcut, int ncutprob, int64_t ncutblk, int j) {
  if (ncutblk > 0) {
    fcw_status st = launch_cut(owner, owner.stream, dcut, ncutprob, nullptr, ncutblk, j);
    if (st) return st;
  }
  return fn(owner.stream, dprobs, ditems, nitems, j, nullptr, 0);
}

bool groupable_2d(const Ctx& a, const Ctx& b) {
  return a.dim == 2 && b.dim == 2 && a.ncomp == 1 && b.ncomp == 1 && a.p == b.p &&
         a.precision == b.precision && a.precision != FCW_BF16;
}

// A batched group: the first member's configuration choice gives the 2-D kernel (its tile
// shape applies to every member); one launch per step over all members' items.
fcw_status run_group(Ctx& owner, const std::vector<GroupMember>& m, bool graph,
                     const StepHook* hook) {
  const int fp64 = owner.precision == FCW_FP64;
  StepCand sc;
  step_candidates(owner, owner.tile_choice, &sc);
  if (!sc.f2d) step_candidates(owner, 0, &sc);
  if (!sc.f2d) {
    set_error("batched runs need 2-D scalar problems");
    return FCW_E_UNSUPPORTED;
  }
  const size_t rs = prob2d_size(fp64);
  const size_t cs = cutprob_size(fp64);
  std::vector<char> rec(rs * m.size()), cut;
  std::vector<int4> items;
  int nmax = 0, ncutprob = 0;
  int64_t ncutblk = 0;
  for (size_t i = 0; i < m.size(); ++i) {
    const GroupMember& g = m[i];
    Ctx& c = *g.ctx;
    if (g.nsteps <= 0) continue;
    fcw_status st = ensure_ycut(c, g.nrhs);
    if (st) return st;
    if (c.n_cut_cand > 0) {
      cut.resize(cs * (ncutprob + 1));
      ncutblk += cutprob_fill(c, cut.data() + cs * ncutprob, g.u, g.scratch, g.nrhs, g.nsteps,
                              ncutblk);
      ++ncutprob;
    }
    if (g.nsteps % 2 == 1)
      FCW_HIP(hipMemcpyAsync(g.scratch, g.u, (size_t)g.nrhs * c.ndof * c.state_bytes(),
                             hipMemcpyDeviceToDevice, owner.stream));
    prob2d_fill(c, rec.data() + rs * i, g.u, g.scratch, g.d, g.t0, g.dt, g.nsteps, g.start,
                sc.tile[0], sc.tile[1], c.d_src);
    const int ntx = (c.ncells[0] + sc.tile[0] - 1) / sc.tile[0];
    const int nty = (c.ncells[1] + sc.tile[1] - 1) / sc.tile[1];
    for (int t = 0; t < ntx * nty; ++t)
      for (int r = 0; r < g.nrhs; ++r) items.push_back(make_int4((int)i, r, t, 0));
    nmax = std::max(nmax, g.nsteps);
  }
  if (items.empty()) return FCW_OK;
  // work list in device memory: 2-D records, items, cut-cell records
  std::vector<char> host(rec.size() + items.size() * sizeof(int4) + cut.size());
  std::memcpy(host.data(), rec.data(), rec.size());
  std::memcpy(host.data() + rec.size(), items.data(), items.size() * sizeof(int4));
  if (!cut.empty())
    std::memcpy(host.data() + rec.size() + items.size() * sizeof(int4), cut.data(), cut.size());
  fcw_status st = stage_worklist(owner, host.data(), host.size());
  if (st) return st;
  const int nitems = (int)items.size();
  const int4* ditems = (const int4*)((char*)owner.d_wl + rec.size());
  const void* dcut = (const char*)owner.d_wl + rec.size() + items.size() * sizeof(int4);
  if (!graph || hook) {
    if (hook && (st = hook->fn(hook->arg, owner.stream, -1))) return st;
    for (int j = 0; j < nmax; ++j) {
      if ((st = group_step(owner, sc.f2d, owner.d_wl, ditems, nitems, dcut, ncutprob, ncutblk, j)))
        return st;
      if (hook && (st = hook->fn(hook->arg, owner.stream, j))) return st;
    }
    return FCW_OK;
  }
  // graph replay: the records live in device memory, so a cached graph stays valid for
  // the same kernels, work-list buffer and layout (member records, items and cut-cell
  // records at the same offsets), cut-block count and step count
  const int nprob = (int)m.size();
  if (!(owner.graph_exec && owner.graph_fn == (const void*)sc.f2d &&
        owner.graph_nitems == nitems && owner.graph_nsteps == nmax &&
        owner.graph_ncut == ncutblk && owner.graph_wl == owner.d_wl &&
        owner.graph_nprob == nprob && owner.graph_ncutprob == ncutprob)) {
    if (owner.graph_exec) FCW_HIP(hipGraphExecDestroy(owner.graph_exec));
    owner.graph_exec = nullptr;
    hipGraph_t g = nullptr;
    FCW_HIP(hipStreamBeginCapture(owner.stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < nmax && st == FCW_OK; ++j)
      st = group_step(owner, sc.f2d, owner.d_wl, ditems, nitems, dcut, ncutprob, ncutblk, j);
    hipError_t e = hipStreamEndCapture(owner.stream, &g);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&owner.graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    owner.graph_fn = (const void*)sc.f2d;
    owner.graph_nitems = nitems;
    owner.graph_nsteps = nmax;
    owner.graph_ncut = ncutblk;
    owner.graph_wl = owner.d_wl;
    owner.graph_nprob = nprob;
    owner.graph_ncutprob = ncutprob;
  }
  FCW_HIP(hipGraphLaunch(owner.graph_exec, owner.stream));
  return FCW_OK;
}

bool groupable_3d(const Ctx& a, const Ctx& b) {
  return a.dim == 3 && b.dim == 3 && a.ncomp == b.ncomp && a.p == b.p &&
         a.precision == b.precision;
}

// A batched group of 3-D problems of one kind: the owner's step configuration (kernel and
// tile shape) for every member; the resident blocks of that kernel are shared out in
// proportion to the members' tiles (at least one per XCD each), and every launch walks
// each member's tiles with its own share.  One cut-cell launch and one step launch per
// step cover all members.
fcw_status run_group3d(Ctx& owner, const std::vector<GroupMember>& m, bool graph,
                       const StepHook* hook) {
  const bool fp64 = owner.precision == FCW_FP64;
  Cand cs[kMaxCand];
  const int nc = cands_for(owner, fp64, cs);
  if (nc == 0) {
    set_error("no step kernel built for this 3-D kind");
    return FCW_E_UNSUPPORTED;
  }
  int choice = owner.tile_choice;
  if (choice < 0 || choice >= nc) choice = 0;
  const BatchOps* ops = cs[choice].ops;
  const size_t rs = ops->rec_size;
  const size_t cps = cutprob_size(fp64);
  std::vector<const GroupMember*> act;
  int64_t tiles_total = 0;
  for (const GroupMember& g : m)
    if (g.nsteps > 0) {
      act.push_back(&g);
      tiles_total += ops->ntiles(*g.ctx);
    }
  if (act.empty()) return FCW_OK;
  const int nprob = (int)act.size();
  const int per_xcd = std::max(1, ops->blocks_per_xcd());
  std::vector<char> rec(rs * nprob), cut;
  std::vector<int32_t> bstart(nprob + 1, 0);
  int maxrhs = 1, nmax = 0, ncutprob = 0;
  int64_t ncutblk = 0;
  for (int i = 0; i < nprob; ++i) {
    const GroupMember& g = *act[i];
    Ctx& c = *g.ctx;
    fcw_status st = ensure_ycut(c, g.nrhs);
    if (st) return st;
    if (c.n_cut_cand > 0) {
      cut.resize(cps * (ncutprob + 1));
      ncutblk += cutprob_fill(c, cut.data() + cps * ncutprob, g.u, g.scratch, g.nrhs, g.nsteps,
                              ncutblk);
      ++ncutprob;
    }
    if (g.nsteps % 2 == 1)
      FCW_HIP(hipMemcpyAsync(g.scratch, g.u, (size_t)g.nrhs * c.ndof * c.state_bytes(),
                             hipMemcpyDeviceToDevice, owner.stream));
    ops->fill(c, rec.data() + rs * i, g.u, g.scratch, g.d, g.t0, g.dt, g.nsteps, g.start,
              g.nrhs);
    const int nt = ops->ntiles(c);
    const int chunk = (nt + 7) / 8;
    const int share = (int)((int64_t)per_xcd * nt / std::max<int64_t>(tiles_total, 1));
    const int nbx = std::max(1, std::min(chunk, share));
    bstart[i + 1] = bstart[i] + 8 * nbx;
    maxrhs = std::max(maxrhs, g.nrhs);
    nmax = std::max(nmax, g.nsteps);
  }
  const int nblocks = bstart[nprob];
  // work list: records, block starts (padded to 16 bytes), cut-cell records
  const size_t bs_bytes = ((bstart.size() * sizeof(int32_t)) + 15) / 16 * 16;
  std::vector<char> host(rec.size() + bs_bytes + cut.size(), 0);
  std::memcpy(host.data(), rec.data(), rec.size());
  std::memcpy(host.data() + rec.size(), bstart.data(), bstart.size() * sizeof(int32_t));
  if (!cut.empty()) std::memcpy(host.data() + rec.size() + bs_bytes, cut.data(), cut.size());
  fcw_status st = stage_worklist(owner, host.data(), host.size());
  if (st) return st;
  const int32_t* dbs = (const int32_t*)((char*)owner.d_wl + rec.size());
  const void* dcut = (const char*)owner.d_wl + rec.size() + bs_bytes;
  auto step = [&](int j) -> fcw_status {
    if (ncutblk > 0) {
      fcw_status s2 = launch_cut(owner, owner.stream, dcut, ncutprob, nullptr, ncutblk, j);
      if (s2) return s2;
    }
    return ops->run(owner.stream, owner.d_wl, dbs, nprob, nblocks, maxrhs, j);
  };
  if (!graph || hook) {
    if (hook && (st = hook->fn(hook->arg, owner.stream, -1))) return st;
    for (int j = 0; j < nmax; ++j) {
      if ((st = step(j))) return st;
      if (hook && (st = hook->fn(hook->arg, owner.stream, j))) return st;
    }
    return FCW_OK;
  }
  // graph replay, cached while the kernels, the work-list buffer and its layout, the
  // cut-block count and the step count stay the same
  if (!(owner.graph_exec && owner.graph_fn == (const void*)ops &&
        owner.graph_nitems == nblocks && owner.graph_nsteps == nmax &&
        owner.graph_ncut == ncutblk && owner.graph_wl == owner.d_wl &&
        owner.graph_nprob == nprob && owner.graph_ncutprob == ncutprob)) {
    if (owner.graph_exec) FCW_HIP(hipGraphExecDestroy(owner.graph_exec));
    owner.graph_exec = nullptr;
    hipGraph_t gr = nullptr;
    FCW_HIP(hipStreamBeginCapture(owner.stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < nmax && st == FCW_OK; ++j) st = step(j);
    hipError_t e = hipStreamEndCapture(owner.stream, &gr);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&owner.graph_exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    owner.graph_fn = (const void*)ops;
    owner.graph_nitems = nblocks;
    owner.graph_nsteps = nmax;
    owner.graph_ncut = ncutblk;
    owner.graph_wl = owner.d_wl;
    owner.graph_nprob = nprob;
    owner.graph_ncutprob = ncutprob;
  }
  FCW_HIP(hipGraphLaunch(owner.graph_exec, owner.stream));
  return FCW_OK;
}

// Advance nrhs right-hand sides by nsteps steps with configuration `choice`; the final
// state is in u.  `scratch` holds nrhs*ndof state words.
fcw_status run_steps(Ctx& c, int choice, int nrhs, void* u, void* d, void* scratch, double t0,
                     double dt, int nsteps, int start, const StepHook* hook) {
  if (nsteps <= 0) return FCW_OK;
  if (hook) {
    fcw_status st = hook->fn(hook->arg, c.stream, -1);
    if (st) return st;
  }
  const size_t bytes = (size_t)nrhs * c.ndof * c.state_bytes();
  StepCand sc;
  const int n = step_candidates(c, choice, &sc);
  if (choice < 0 || choice >= n) step_candidates(c, 0, &sc);
  if (nsteps % 2 == 1) FCW_HIP(hipMemcpyAsync(scratch, u, bytes, hipMemcpyDeviceToDevice, c.stream));
  if (sc.f2d) {
    const int fp64 = c.precision == FCW_FP64;
    fcw_status st = ensure_ycut(c, nrhs);
    if (st) return st;
    char crec[256];
    const int64_t ncutblk = cutprob_fill(c, crec, u, scratch, nrhs, nsteps, 0);
    const int ntx = (c.ncells[0] + sc.tile[0] - 1) / sc.tile[0];
    const int nty = (c.ncells[1] + sc.tile[1] - 1) / sc.tile[1];
    alignas(16) char rec[256];
    if (prob2d_size(fp64) > sizeof rec) {
      set_error("2-D problem record larger than its buffer");
      return FCW_E_DEVICE;
    }
    prob2d_fill(c, rec, u, scratch, d, t0, dt, nsteps, start, sc.tile[0], sc.tile[1], c.d_src);
    // one problem: its record goes by value, items are implicit (tile-major, rhs fastest)
    const int nitems = ntx * nty * nrhs;
    for (int j = 0; j < nsteps; ++j) {
      if (c.n_cut_cand > 0 && !c.skip_cut &&
          (st = launch_cut(c, c.stream, nullptr, 1, crec, ncutblk, j)))
        return st;
      if ((st = sc.f2d(c.stream, nullptr, nullptr, nitems, j, rec, nrhs))) return st;
      if (hook && (st = hook->fn(hook->arg, c.stream, j))) return st;
    }
    return FCW_OK;
  }
  void* a = (nsteps % 2 == 1) ? scratch : u;
  void* b = (nsteps % 2 == 1) ? u : scratch;
  for (int j = 0; j < nsteps; ++j) {
    fcw_status st = sc.fgen(c, kModeStep, nrhs, a, b, d, t0 + j * dt, dt, (start && j == 0) ? 1 : 0);
    if (st) return st;
    if (hook && (st = hook->fn(hook->arg, c.stream, j))) return st;
    void* t = a;
    a = b;
    b = t;
  }
  return FCW_OK;
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
