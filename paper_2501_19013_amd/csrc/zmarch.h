// 3-D step kernel that marches in z (the central-difference step of eq. cdm with the
// element-by-element K u of eq. semi), so no cell layer is multiplied twice:
//
//  * A block owns the cells of an x-y tile of TX x TY cells over ZR cell layers (an item),
//    plus one ring of cells on the low x and y sides.  It walks the layers bottom to top;
//    the layer below its first one is the only extra layer it multiplies.
//  * The node values of a layer (its P + 1 node planes over the tile and the ring) are
//    staged global -> LDS by range-checked buffer loads with an LDS destination (planes
//    and nodes outside the grid read zero); the next layer's planes, cell infos, d and
//    stored inverse masses are in flight while the current layer is multiplied and
//    updated.  The cut-cell products of a layer (cut-cell kernel) are copied first, so
//    the wait after the products covers them with a fixed count of later loads.
//  * Products: the uncut cells of the layer are compacted into a list and multiplied in
//    batches of 16 on the matrix cores (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64,
//    K_ref rows as the A operand).  When K_ref has more than 32 fragments per lane, each
//    wave keeps the fragments of one 16-row block of K_ref in registers and walks the
//    batches with it.  Cells outside the domain get zero rows, cut cells their copies.
//  * Each owned node of the layer's lower P planes gathers its (at most 8) cells' results
//    in the order of the tile kernel (lower z first, then lower y, lower x; the lower
//    layer's top-plane products are kept from the previous layer) and applies the
//    lumped-mass update in increment form; the arithmetic is that of the tile kernel,
//    operation for operation, so both give the same bits.  The top node plane of the
//    grid is updated after the last layer.
//  * Stores are buffer stores with an out-of-range offset for units that own no node, so
//    each wave issues a fixed number per layer and the end-of-layer wait leaves exactly
//    those in flight (stores count in vmcnt on this target).
#pragma once

#include "step_common.h"

namespace fcw {

namespace zm {

constexpr uint32_t kNoAccess = 0xFFFFFFF0u;  // out-of-range buffer offset: no access

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0,
                                           (int)(bytes < 0x7FFFFFF0 ? bytes : 0x7FFFFFF0),
                                           0x00020000);
}

// s_waitcnt vmcnt(N), expcnt and lgkmcnt not waited for (gfx9 encoding)
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
  constexpr int imm = (N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(imm);
  asm volatile("" ::: "memory");
}

template <typename T>
__device__ inline T load(__amdgpu_buffer_rsrc_t rs, uint32_t voff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, 0));
  } else {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, 0));
  }
}

template <typename T>
__device__ inline void store(__amdgpu_buffer_rsrc_t rs, uint32_t voff, T v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, voff, 0, 0);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, voff, 0, 0);
  }
}

}  // namespace zm

template <typename T, int P, int NCOMP, int TX, int TY, int ZR, int NW>
__global__ __launch_bounds__(64 * NW, 3) void zmarch_kernel(StepArgs<T> ain) {
  constexpr int NT = 64 * NW;
  constexpr int NP1 = P + 1;
  constexpr int NP2 = NP1 * NP1;
  constexpr int NS = NP2 * NP1;
  constexpr int NL = NCOMP * NS;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  constexpr bool AREG = NMB * NKS <= 32;  // every K_ref fragment in registers
  static_assert(AREG || NW % NMB == 0, "each wave keeps one 16-row block of K_ref");
  constexpr int RCX = TX + 1, RCY = TY + 1, NRC = RCX * RCY;  // region cells of a layer
  static_assert(NRC <= 128, "two cell infos per lane");
  constexpr int RNX = RCX * P + 1, RNY = RCY * P + 1, PLN = RNX * RNY;
  constexpr int DPE = (int)(sizeof(T) / 4);
  constexpr int LAYV = NP1 * NCOMP * PLN;                 // node values of a layer
  constexpr int NCH = (LAYV * DPE + NT - 1) / NT;         // staging loads per wave
  constexpr int LAYD = NCH * NT;                          // dwords of a layer buffer
  constexpr int NLP = NL | 1;                             // product stride per cell
  constexpr int NTOP = NCOMP * NP2;                       // top-plane products per cell
  constexpr int OX = TX * P + 1, OY = TY * P + 1;         // owned node box (at most)
  constexpr int NUP = P * OX * OY;                        // update units of a layer
  constexpr int KU = (NUP + NT - 1) / NT;
  constexpr int KT = (OX * OY + NT - 1) / NT;             // units of the grid's top plane
  static_assert(KT <= KU, "the top plane's units are a prefix of a layer's units");
  constexpr int NFIX = 2 + NCH + KU * (NCOMP + 1);        // loads per wave after the copies
  constexpr int NST = 2 * KU * NCOMP;                     // stores per wave per layer
  static_assert(NFIX + NST < 64, "vmcnt range");

  __shared__ __attribute__((aligned(16))) uint32_t u_l[2][LAYD];  // two layers: [iz][comp][y][x]
  __shared__ __attribute__((aligned(16))) T y_c[NRC * NLP];  // products of the current layer
  __shared__ T y_t[2][NRC * NTOP];   // top-plane products of the current / previous layer
  __shared__ int info_s[NRC];
  __shared__ int list_s[NRC];        // uncut cells of the layer
  __shared__ int olist_s[NRC];       // cells of the layer outside the domain
  __shared__ int cnt_s[2];
  __shared__ double ft_s;
  __shared__ int src_on;

  // ---- the block's problem (batched launches: the record whose block range holds it) ----
  StepArgs<T> a = ain;
  int bx = (int)blockIdx.x, nbk = (int)gridDim.x;
  if (ain.nprob > 0) {
    int pi = 0;
    while (pi + 1 < ain.nprob && ain.bstart[pi + 1] <= bx) ++pi;
    a = ain.probs[pi];
    const int j = ain.jstep;
    if (j >= a.nsteps || (int)blockIdx.y >= a.nrhs) return;
    bx -= ain.bstart[pi];
    nbk = ain.bstart[pi + 1] - ain.bstart[pi];
    T* ua = a.u_out;
    const bool par = ((a.nsteps - 1 - j) & 1) != 0;
    a.u_in = par ? ua : a.u_alt;
    a.u_out = par ? a.u_alt : ua;
    a.t = __dadd_rn(a.t0, __dmul_rn((double)j, a.dt));  // as the host forms t0 + j dt
    a.start = (a.start && j == 0) ? 1 : 0;
  }
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int npx = a.np[0], npy = a.np[1], npz = a.np[2];
  const int ntx = a.ntile[0], nty = a.ntile[1];
  const int64_t roff = (int64_t)rhs * a.ndof;
  const int64_t sbytes = a.ndof * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t urs_in = zm::rsrc(a.u_in + roff, sbytes);
  const __amdgpu_buffer_rsrc_t urs_out = zm::rsrc(a.u_out + roff, sbytes);
  const __amdgpu_buffer_rsrc_t drs = zm::rsrc(a.d + roff, sbytes);
  const __amdgpu_buffer_rsrc_t mrs = zm::rsrc(a.invm, a.nnodes * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t irs =
      zm::rsrc(a.info, (int64_t)nx * ny * nz * (int64_t)sizeof(int32_t));
  const int64_t plane = (int64_t)npx * npy;

  // ---- once per block: K_ref fragments; the B-operand offsets of this lane's k rows ----
  constexpr int NAM = AREG ? NMB : 1;
  const int mbw = AREG ? 0 : wave % NMB;  // this wave's row block (one-block form)
  T areg[NAM][NKS];
#pragma unroll
  for (int m = 0; m < NAM; ++m)
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int r = (AREG ? m : mbw) * 16 + lc, cc = 4 * kk + lk;
      const T v = a.kref[min(r, NL - 1) * NL + min(cc, NL - 1)];
      areg[m][kk] = (r < NL && cc < NL) ? v : T(0);
    }
  // (two 16-bit offsets per register; padded k rows read a real node, the matching K_ref
  // columns being zero)
  static_assert(LAYV < 65536, "16-bit operand offsets");
  constexpr int NKP = (NKS + 1) / 2;
  uint32_t offp[NKP];
#pragma unroll
  for (int q = 0; q < NKP; ++q) {
    uint32_t v = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jj = min(4 * (2 * q + h) + lk, NL - 1);
      const int comp = jj / NS, loc = jj % NS;
      const int ix = loc % NP1, iy = (loc / NP1) % NP1, iz = loc / NP2;
      v |= (uint32_t)(((iz * NCOMP + comp) * RNY + iy) * RNX + ix) << (16 * h);
    }
    offp[q] = v;
  }

  // the source's time function at this step (the same for every item of the block)
  if (tid == 0) ft_s = (a.src != nullptr) ? ricker(a.t, a.src[rhs].f0) : 0.0;

  const int nitems = a.ntiles;
  const int nbx = nbk / 8;
  for (int tk = bx / 8; tk < a.chunk; tk += nbx) {
    const int item = (bx % 8) * a.chunk + tk;
    if (item >= nitems) break;
    const int cx0 = (item % ntx) * TX, cy0 = ((item / ntx) % nty) * TY;
    const int cz0 = (item / (ntx * nty)) * ZR, cz1 = min(cz0 + ZR, nz);
    const int rnx0 = (cx0 - 1) * P, rny0 = (cy0 - 1) * P;
    const int ox0 = cx0 * P, oy0 = cy0 * P;
    const int onx = (cx0 + TX >= nx) ? npx - ox0 : TX * P;
    const int ony = (cy0 + TY >= ny) ? npy - oy0 : TY * P;

    // ---- loads of layer l: infos (raw value + in-grid flag), node planes, update operands
    int inf_raw[2];
    bool inf_in[2];
    auto load_info = [&](int l) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = lane + 64 * h;
        const int gx = cx0 - 1 + c % RCX, gy = cy0 - 1 + c / RCX;
        const bool in = c < NRC && gx >= 0 && gx < nx && gy >= 0 && gy < ny && l >= 0 && l < nz;
        const int64_t cell = gx + (int64_t)nx * (gy + (int64_t)ny * l);
        inf_raw[h] = (int)__builtin_amdgcn_raw_buffer_load_b32(
            irs, in ? (uint32_t)(cell * 4) : zm::kNoAccess, 0, 0);
        inf_in[h] = in;
      }
    };
    auto stage_layer = [&](int l, uint32_t* dst) {
      // not unrolled: the per-lane offsets are recomputed rather than held in registers
#pragma unroll 1
      for (int ch = 0; ch < NCH; ++ch) {
        const int dw = (ch * NW + wave) * 64 + lane;
        const int e = dw / DPE, half = dw % DPE;
        const int pc = e / PLN, w = e - pc * PLN;
        const int iz = pc / NCOMP, comp = pc - iz * NCOMP;
        const int ry = w / RNX, rx = w - ry * RNX;
        const int gz = l * P + iz, gy = rny0 + ry, gx = rnx0 + rx;
        const bool in = e < LAYV && gx >= 0 && gx < npx && gy >= 0 && gy < npy && gz >= 0 &&
                        gz < npz;
        const int64_t byte =
            ((int64_t)comp * a.nnodes + gx + npx * (int64_t)gy + plane * gz) * (int64_t)sizeof(T) +
            4 * half;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            urs_in, (__attribute__((address_space(3))) void*)(dst + (ch * NW + wave) * 64), 4,
            in ? (uint32_t)byte : zm::kNoAccess, 0, 0, 0);
      }
    };
    T d_c[KU][NCOMP], d_n[KU][NCOMP], m_c[KU], m_n[KU];
    // unit u of layer l: local plane u / (OX OY), then y, then x; layer nz holds only the
    // grid's top plane, and layers at or above the item's end belong to the next item
    auto load_upd = [&](int l) {
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const int u = tid + NT * k;
        const int lz = u / (OX * OY), ly = (u / OX) % OY, lx = u % OX;
        const bool own = u < NUP && lx < onx && ly < ony && l >= cz0 &&
                         (l < cz1 || (l == nz && lz == 0));
        const int64_t node = (ox0 + lx) + npx * (int64_t)(oy0 + ly) + plane * (l * P + lz);
        m_n[k] = zm::load<T>(mrs, own ? (uint32_t)(node * (int64_t)sizeof(T)) : zm::kNoAccess);
#pragma unroll
        for (int comp = 0; comp < NCOMP; ++comp)
          d_n[k][comp] = zm::load<T>(
              drs, own ? (uint32_t)((comp * a.nnodes + node) * (int64_t)sizeof(T))
                       : zm::kNoAccess);
      }
    };

    // ---- item prologue: does the source touch the item; the ring layer's loads ----
    if (tid == 0) {
      src_on = 0;
      if (a.src != nullptr) {
        const SourceDev& s = a.src[rhs];
        // owned node box of the item vs node box of the source cell
        const int o0[3] = {ox0, oy0, cz0 * P};
        const int o1[3] = {ox0 + onx, oy0 + ony, (cz1 >= nz) ? npz : cz1 * P};
        bool hit = true;
        for (int k = 0; k < 3; ++k)
          if (s.cell[k] * P + P < o0[k] || s.cell[k] * P >= o1[k]) hit = false;
        src_on = hit ? 1 : 0;
      }
    }
    load_info(cz0 - 1);
    stage_layer(cz0 - 1, u_l[(cz0 - 1) & 1]);
    load_upd(cz0 - 1);  // owns nothing: keeps the per-layer load count fixed
    zm::wait_vmcnt<0>();
    block_sync();

    for (int l = cz0 - 1; l < cz1; ++l) {
      const bool ring = l < cz0;
      const int bl = l & 1;
      // ---- A1: this layer's infos and lists (loaded one layer ahead) ----
      int inf_c[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) inf_c[h] = inf_in[h] ? inf_raw[h] : kInfoOut;
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        m_c[k] = m_n[k];
#pragma unroll
        for (int comp = 0; comp < NCOMP; ++comp) d_c[k][comp] = d_n[k][comp];
      }
      if (wave == 0) {
        int nu = 0, no = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = lane + 64 * h;
          const bool valid = c < NRC;
          if (valid) info_s[c] = inf_c[h];
          const unsigned long long below = (1ull << lane) - 1ull;
          const unsigned long long mu = __ballot(valid && inf_c[h] == kInfoUncut);
          const unsigned long long mo = __ballot(valid && inf_c[h] == kInfoOut);
          if (valid && inf_c[h] == kInfoUncut) list_s[nu + __popcll(mu & below)] = c;
          if (valid && inf_c[h] == kInfoOut) olist_s[no + __popcll(mo & below)] = c;
          nu += __popcll(mu);
          no += __popcll(mo);
        }
        if (lane == 0) {
          cnt_s[0] = nu;
          cnt_s[1] = no;
        }
      }
      block_sync();

      // ---- A2: the cut-cell copies of this layer, then the next layer's loads ----
      {
        constexpr int RDW = NL * DPE;
        int seen = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c0 = 64 * h;
          const int cq = c0 + lane;
          unsigned long long mask = __ballot(cq < NRC && info_s[min(cq, NRC - 1)] >= 0);
          while (mask) {
            const int bit = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if ((seen++ % NW) != wave) continue;
            const int c = c0 + bit;
            const uint32_t* src =
                (const uint32_t*)(a.ycut + ((int64_t)rhs * a.ncand + info_s[c]) * NL);
            uint32_t* dst = (uint32_t*)(y_c + c * NLP);
#pragma unroll
            for (int ch = 0; ch < (RDW + 63) / 64; ++ch)
              if (ch * 64 + lane < RDW)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void*)(src + ch * 64 + lane),
                    (__attribute__((address_space(3))) void*)(dst + ch * 64), 4, 0, 0);
          }
        }
      }
      // nothing below moves above the copies (the wait after the products counts on it)
      asm volatile("" ::: "memory");
      load_info(l + 1);
      stage_layer(l + 1, u_l[bl ^ 1]);
      load_upd(l + 1);

      // ---- B: products of the layer's uncut cells; zero rows of its outside cells ----
      {
        const int nu = cnt_s[0], no = cnt_s[1];
        const int nbat = (nu + 15) / 16;
        const T* ub = (const T*)u_l[bl];
        auto batch = [&](int b, int m0, int m1) {
          const int slot = b * 16 + lc;
          const int cl = list_s[min(slot, nu - 1)];
          const int base = (cl % RCX) * P + (cl / RCX) * P * RNX;
          // operands in two halves (fewer live registers); each half's loads are issued
          // before its products
          constexpr int KH = AREG ? NKS : (NKS + 1) / 2;
          T bv[NKS];
          typename Mma<T>::acc acc[NAM];
#pragma unroll
          for (int m = 0; m < NAM; ++m) acc[m] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
          for (int k0 = 0; k0 < NKS; k0 += KH) {
#pragma unroll
            for (int kk = k0; kk < k0 + KH && kk < NKS; ++kk)
              bv[kk] = ub[base + (int)((offp[kk / 2] >> (16 * (kk % 2))) & 0xFFFFu)];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < NAM; ++m) {
              if (m < m0 || m >= m1) continue;
#pragma unroll
              for (int kk = k0; kk < k0 + KH && kk < NKS; ++kk)
                acc[m] = Mma<T>::mma(areg[m][kk], bv[kk], acc[m]);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int m = 0; m < NAM; ++m) {
            if (m < m0 || m >= m1) continue;
            const int mb = AREG ? m : mbw;
            if (slot < nu) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = mb * 16 + Mma<T>::row(lk, r);
                if (i < NL) y_c[cl * NLP + i] = acc[m][r];
              }
            }
          }
        };
        if constexpr (AREG) {
          for (int b = wave; b < nbat; b += NW) batch(b, 0, NAM);
        } else {
          for (int b = wave / NMB; b < nbat; b += NW / NMB) batch(b, 0, 1);
        }
        for (int i = tid; i < no * NL; i += NT) y_c[olist_s[i / NL] * NLP + i % NL] = T(0);
      }
      zm::wait_vmcnt<NFIX>();  // this layer's cut-cell copies are done
      block_sync();

      // ---- C: gather and update of the owned nodes of planes l P .. l P + P - 1 ----
      const T* yt_prev = y_t[bl ^ 1];
      if (!ring) {
        const T* ub = (const T*)u_l[bl];
        // an opaque zero that changes every layer: the gather's addresses are recomputed
        // per layer instead of being held in registers across the march
        int zo = 0;
        asm volatile("" : "+v"(zo) : "s"(l));
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          const int u = tid + NT * k + zo;
          const int lz = min(u / (OX * OY), P - 1), ly = (u / OX) % OY, lx = u % OX;
          const bool own = u < NUP && lx < onx && ly < ony;
          const int gx = ox0 + lx, gy = oy0 + ly, gz = l * P + lz;
          // cells around the node along x and y (region-local), as in the tile kernel
          const int qx = gx / P, remx = gx - qx * P;
          const int qy = gy / P, remy = gy - qy * P;
          const bool uax = remx == 0 && gx > 0, ubx = gx < nx * P;
          const bool uay = remy == 0 && gy > 0, uby = gy < ny * P;
          const int cax = max(qx - cx0, 0), cbx = min(qx - cx0 + 1, RCX - 1);
          const int cay = max(qy - cy0, 0), cby = min(qy - cy0 + 1, RCY - 1);
          const bool uaz = lz == 0 && gz > 0;
          T r[NCOMP];
#pragma unroll
          for (int comp = 0; comp < NCOMP; ++comp) r[comp] = T(0);
#pragma unroll
          for (int sz = 0; sz < 2; ++sz)
#pragma unroll
            for (int sy = 0; sy < 2; ++sy)
#pragma unroll
              for (int sx = 0; sx < 2; ++sx) {
                const bool use = (sx ? ubx : uax) && (sy ? uby : uay) && (sz ? true : uaz);
                const int cell = (sx ? cbx : cax) + RCX * (sy ? cby : cay);
                const int lxx = sx ? remx : P, lyy = sy ? remy : P;
#pragma unroll
                for (int comp = 0; comp < NCOMP; ++comp) {
                  const T v = sz ? y_c[cell * NLP + comp * NS + lxx + NP1 * (lyy + NP1 * lz)]
                                 : yt_prev[cell * NTOP + comp * NP2 + lxx + NP1 * lyy];
                  r[comp] += use ? v : T(0);
                }
              }
          int sloc = -1;
          if (src_on) {
            const SourceDev& s = a.src[rhs];
            const int sx = gx - s.cell[0] * P, sy = gy - s.cell[1] * P, sz = gz - s.cell[2] * P;
            if (sx >= 0 && sx <= P && sy >= 0 && sy <= P && sz >= 0 && sz <= P)
              sloc = sx + NP1 * (sy + NP1 * sz);
          }
          const int64_t node = gx + npx * (int64_t)gy + plane * gz;
          const int rl = (gx - rnx0) + RNX * (gy - rny0);
#pragma unroll
          for (int comp = 0; comp < NCOMP; ++comp) {
            T F = T(0);
            if (sloc >= 0) F = (T)(ft_s * a.src[rhs].b[comp * NS + sloc]);
            T acc = a.dt2 * m_c[k] * (F - r[comp]);
            if (a.start) acc = acc * T(0.5);
            const T dn = d_c[k][comp] + acc;
            const T un = ub[(lz * NCOMP + comp) * PLN + rl] + dn;
            const uint32_t vo =
                own ? (uint32_t)((comp * a.nnodes + node) * (int64_t)sizeof(T)) : zm::kNoAccess;
            zm::store<T>(drs, vo, dn);
            zm::store<T>(urs_out, vo, un);
          }
          __builtin_amdgcn_sched_barrier(0);  // one unit's gather at a time (registers)
        }
      }
      // top-plane products of this layer, for the layer above
      for (int i = tid; i < NRC * NTOP; i += NT) {
        const int c = i / NTOP, rr = i % NTOP;
        const int comp = rr / NP2, w = rr % NP2;
        y_t[bl][i] = y_c[c * NLP + comp * NS + P * NP2 + w];
      }
      if (!ring) zm::wait_vmcnt<NST>();  // the next layer's loads are done
      else zm::wait_vmcnt<0>();
      block_sync();
    }

    // ---- the top node plane of the grid: only the layer below contributes ----
    if (cz1 == nz) {
      const int lb = (nz - 1) & 1;
      const T* yt = y_t[lb];
      const T* ub = (const T*)u_l[lb];
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int u = tid + NT * k;
        const int ly = (u / OX) % OY, lx = u % OX;
        const bool own = u < OX * OY && lx < onx && ly < ony;
        const int gx = ox0 + lx, gy = oy0 + ly, gz = nz * P;
        const int qx = gx / P, remx = gx - qx * P;
        const int qy = gy / P, remy = gy - qy * P;
        const bool uax = remx == 0 && gx > 0, ubx = gx < nx * P;
        const bool uay = remy == 0 && gy > 0, uby = gy < ny * P;
        const int cax = max(qx - cx0, 0), cbx = min(qx - cx0 + 1, RCX - 1);
        const int cay = max(qy - cy0, 0), cby = min(qy - cy0 + 1, RCY - 1);
        T r[NCOMP];
#pragma unroll
        for (int comp = 0; comp < NCOMP; ++comp) r[comp] = T(0);
        // the tile kernel's order with the upper z cells (outside the grid) adding zeros
#pragma unroll
        for (int sz = 0; sz < 2; ++sz)
#pragma unroll
          for (int sy = 0; sy < 2; ++sy)
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
              const bool use = (sx ? ubx : uax) && (sy ? uby : uay) && sz == 0;
              const int cell = (sx ? cbx : cax) + RCX * (sy ? cby : cay);
              const int lxx = sx ? remx : P, lyy = sy ? remy : P;
#pragma unroll
              for (int comp = 0; comp < NCOMP; ++comp) {
                const T v = yt[cell * NTOP + comp * NP2 + lxx + NP1 * lyy];
                r[comp] += use ? v : T(0);
              }
            }
        int sloc = -1;
        if (src_on) {
          const SourceDev& s = a.src[rhs];
          const int sx = gx - s.cell[0] * P, sy = gy - s.cell[1] * P, sz = gz - s.cell[2] * P;
          if (sx >= 0 && sx <= P && sy >= 0 && sy <= P && sz >= 0 && sz <= P)
            sloc = sx + NP1 * (sy + NP1 * sz);
        }
        const int64_t node = gx + npx * (int64_t)gy + plane * gz;
        const int rl = (gx - rnx0) + RNX * (gy - rny0);
#pragma unroll
        for (int comp = 0; comp < NCOMP; ++comp) {
          T F = T(0);
          if (sloc >= 0) F = (T)(ft_s * a.src[rhs].b[comp * NS + sloc]);
          T acc = a.dt2 * m_n[k] * (F - r[comp]);
          if (a.start) acc = acc * T(0.5);
          const T dn = d_n[k][comp] + acc;
          const T un = ub[(P * NCOMP + comp) * PLN + rl] + dn;
          const uint32_t vo =
              own ? (uint32_t)((comp * a.nnodes + node) * (int64_t)sizeof(T)) : zm::kNoAccess;
          zm::store<T>(drs, vo, dn);
          zm::store<T>(urs_out, vo, un);
        }
      }
    }
    block_sync();  // the next item reuses the LDS
  }
}

}  // namespace fcw
