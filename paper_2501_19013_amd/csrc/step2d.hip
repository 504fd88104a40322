// Central-difference step (paper eq. cdm) for 2-D scalar problems, shaped for CDNA4 wave64:
//
//  * A tile is TX = 64 / P cells wide, so one owned node row of a tile is exactly one
//    wave (lane = x); TY cells high.  A workgroup (4 waves) stages the node values of
//    the tile plus one ring of cells on the low side in LDS, one region row per
//    buffer_load ... lds pair (no VGPRs, out-of-range lanes read zero).
//  * The cells of the region are visited in 4 colour classes (cell parity in x and y).
//    Within a class no two cells share a node, so the element results go straight
//    into an LDS node accumulator with plain read-add-write (no two lanes or waves of
//    a class touch the same node, and every add rounds to nearest); the classes are ordered
//    by barriers, so every node sums its (at most 4) cell contributions in a fixed
//    order: bitwise reproducible, no atomics to global memory, no gather pass.
//  * Uncut cells of a class: 16 per wave on the matrix cores, Y = K_ref [u_e1..u_e16]
//    (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64; K_ref fragments held in VGPRs).
//    Cut cells of a class: one wave per cell streaming its packed K_e, accumulated in
//    FP64 whatever the state precision.
//  * The update d_{k+1} = d_k + dt^2 M^{-1}(F_k - K u_k), u_{k+1} = u_k + d_{k+1} runs
//    row by row (lane = x), with d and M^{-1} prefetched at kernel entry.
#include "step_common.h"

namespace fcw {

template <typename T>
__device__ static inline void buffer_dword_to_lds(__amdgpu_buffer_rsrc_t rsrc, int voffset,
                                                  void* lds_wave_base) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)lds_wave_base,
                                           4, voffset, 0, 0, 0);
}

template <typename T, int P, int TY>
__global__ __launch_bounds__(256) void step2d_kernel(StepArgs<T> a) {
  constexpr int NP1 = P + 1;
  constexpr int NL = NP1 * NP1;
  constexpr int NMB = (NL + 15) / 16;
  constexpr int NKS = (NL + 3) / 4;
  constexpr int NPK = NL * (NL + 1) / 2;
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
  __shared__ int info_s[NRC];
  __shared__ double ft_s;
  __shared__ int src_on;

  const int tile = (int)(blockIdx.x % 8) * a.chunk + (int)(blockIdx.x / 8);
  if (tile >= a.ntiles) return;
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  const int tx = tile % a.ntile[0], ty = tile / a.ntile[0];
  const int cx0 = tx * TX, cy0 = ty * TY;
  const int rcx0 = cx0 - 1, rcy0 = cy0 - 1;
  const int rnx0 = rcx0 * P, rny0 = rcy0 * P;
  const int npx = a.np[0], npy = a.np[1];
  const int ox0 = cx0 * P, oy0 = cy0 * P;
  const int onx = (cx0 + TX >= a.n[0]) ? npx - ox0 : OWX;  // OWX + 1 on the last full tile
  const int ony = (cy0 + TY >= a.n[1]) ? npy - oy0 : TY * P;
  const int64_t roff = (int64_t)rhs * a.ndof;
  const T* uin = a.u_in + roff;
  T* dst_d = a.d + roff;
  T* dst_u = a.u_out + roff;
  const uint32_t nbytes = (uint32_t)(a.nnodes * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ursrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)uin, (short)0, (int)nbytes, 0x00020000);

  // ---- entry: issue every load of the tile ----
  T areg[NMB][NKS];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int kk = 0; kk < NKS; ++kk) {
      const int r = mb * 16 + lc, cc = 4 * kk + lk;
      const T v = a.kref[min(r, NL - 1) * NL + min(cc, NL - 1)];
      areg[mb][kk] = (r < NL && cc < NL) ? v : T(0);
    }
  int inf_r[NCI];
#pragma unroll
  for (int it = 0; it < NCI; ++it) {
    const int c = tid + it * 256;
    const int gx = rcx0 + c % RCX, gy = rcy0 + c / RCX;
    const bool in = c < NRC && gx >= 0 && gx < a.n[0] && gy >= 0 && gy < a.n[1];
    const int v = a.info[in ? gx + a.n[0] * gy : 0];
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
  T d_r[NRW], im_r[NRW];
#pragma unroll
  for (int k = 0; k < NRW; ++k) {
    const int oy = wave + 4 * k;
    const bool own = oy < ony && lane < min(onx, OWX);
    const uint32_t node = own ? (uint32_t)((oy0 + oy) * npx + ox0 + lane) : 0u;
    d_r[k] = dst_d[node];
    im_r[k] = a.invm[node];
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
    if (a.src != nullptr) {
      const SourceDev& s = a.src[rhs];
      const int sx0 = s.cell[0] * P, sy0 = s.cell[1] * P;
      if (sx0 + P >= ox0 && sx0 < ox0 + onx && sy0 + P >= oy0 && sy0 < oy0 + ony) {
        src_on = 1;
        ft_s = ricker(a.t, s.f0);
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
      T bv[NKS];
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk) {
        const T v = u_s[base + offk[kk]];
        bv[kk] = (valid && 4 * kk + lk < NL) ? v : T(0);
      }
      typename Mma<T>::acc acc[NMB];
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) acc[mb] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[mb] = Mma<T>::mma(areg[mb][kk], bv[kk], acc[mb]);
      if (valid) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = mb * 16 + Mma<T>::row(lk, r);
            if (i < NL) r_s[base + (i % NP1) + (i / NP1) * W] += acc[mb][r];
          }
      }
    }
    // cut cells of the class: one wave per cell, lanes = rows of K_e
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
        const T* K = a.kcut + (int64_t)q * NPK;
        const int i = min(lane, NL - 1);
        // FP64 accumulation: the rows of a cut-cell matrix cancel strongly and the
        // small lumped masses of cut-cell nodes amplify any error in their sum
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          const int kidx = (i <= j) ? j * (j + 1) / 2 + i : i * (i + 1) / 2 + j;
          y += (double)K[kidx] * (double)u_s[base + (j % NP1) + (j / NP1) * W];
        }
        if (lane < NL) r_s[base + (i % NP1) + (i / NP1) * W] += (T)y;
      }
    }
    __syncthreads();
  }

  // ---- update, one owned row per wave instruction ----
  const T dt2 = a.dt2;
  const bool half = a.start != 0;
  const SourceDev* src = a.src;
#pragma unroll
  for (int k = 0; k < NRW; ++k) {
    const int oy = wave + 4 * k;
    if (oy >= ony) continue;
    for (int xx = lane; xx < onx; xx += 64) {
      const bool pre = xx < OWX;  // nodes beyond one wave (last column) load here
      const int gx = ox0 + xx, gy = oy0 + oy;
      const uint32_t node = (uint32_t)(gy * npx + gx);
      const int rl = (gx - rnx0) + (gy - rny0) * W;
      T F = T(0);
      if (src_on) {
        const int sx = gx - src[rhs].cell[0] * P, sy = gy - src[rhs].cell[1] * P;
        if (sx >= 0 && sx <= P && sy >= 0 && sy <= P) F = (T)(ft_s * src[rhs].b[sx + NP1 * sy]);
      }
      const T im = pre ? im_r[k] : a.invm[node];
      const T dv = pre ? d_r[k] : dst_d[node];
      T acc = dt2 * im * (F - r_s[rl]);
      if (half) acc = acc * T(0.5);
      const T dn = dv + acc;
      dst_d[node] = dn;
      dst_u[node] = u_s[rl] + dn;
    }
  }
}

template <typename T, int P, int TY>
static fcw_status run2d(Ctx& c, int nrhs, const void* uin, void* uout, void* d, double t,
                        double dt, int start) {
  StepArgs<T> a{};
  constexpr int TX = 64 / P;
  a.info = c.d_info;
  a.kref = (const T*)c.d_kref_s;
  a.kcut = (const T*)c.d_kcut_s;
  a.invm = (const T*)c.d_invm;
  a.n[0] = c.ncells[0];
  a.n[1] = c.ncells[1];
  a.n[2] = 1;
  a.np[0] = c.npts[0];
  a.np[1] = c.npts[1];
  a.np[2] = 1;
  a.ntile[0] = (a.n[0] + TX - 1) / TX;
  a.ntile[1] = (a.n[1] + TY - 1) / TY;
  a.ntile[2] = 1;
  a.ntiles = a.ntile[0] * a.ntile[1];
  a.chunk = (a.ntiles + 7) / 8;
  a.nnodes = c.nnodes;
  a.ndof = c.ndof;
  a.u_in = (const T*)uin;
  a.u_out = (T*)uout;
  a.d = (T*)d;
  a.dt2 = (T)(dt * dt);
  a.start = start;
  a.src = c.d_src;
  a.t = t;
  dim3 grid(8 * a.chunk, nrhs, 1);
  step2d_kernel<T, P, TY><<<grid, 256, 0, c.stream>>>(a);
  FCW_HIP(hipGetLastError());
  return FCW_OK;
}

// 2-D step kernels offered to the autotuner: (P, TY) -> launcher; TX = 64 / P.
using Run2d = fcw_status (*)(Ctx&, int, const void*, void*, void*, double, double, int);

int step2d_candidates(const Ctx& c, int i, Run2d* fn, int tile[3]) {
  if (c.dim != 2 || c.ncomp != 1) return 0;
  struct E { int p, ty; Run2d f32, f64; };
#define FCW_E(PP, TY) E{PP, TY, &run2d<float, PP, TY>, &run2d<double, PP, TY>}
  static const E table[] = {
      FCW_E(1, 16), FCW_E(1, 32), FCW_E(2, 8), FCW_E(2, 16), FCW_E(3, 8), FCW_E(3, 16),
      FCW_E(4, 8), FCW_E(4, 4), FCW_E(4, 16), FCW_E(5, 4), FCW_E(5, 8)};
#undef FCW_E
  int n = 0;
  for (const E& e : table) {
    if (e.p != c.p) continue;
    if (n == i) {
      if (fn) *fn = (c.precision == FCW_FP64) ? e.f64 : e.f32;
      if (tile) { tile[0] = 64 / e.p; tile[1] = e.ty; tile[2] = 1; }
    }
    ++n;
  }
  return n;
}

}  // namespace fcw
