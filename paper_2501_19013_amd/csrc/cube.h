// The rotated cube of the benchmark geometry (Sec. 3.1): the physical domain is the cube
// of half edge a about centre c with axes u_j = column j of T, minus the voids.  Exact
// FP64 predicates with every sum taken left to right in index order (FMA contraction
// off), so that setup and its checks agree bit for bit:
//  * a point is outside iff |l_j| > a for some j, l_j = sum_k (x_k - c_k) T_kj;
//  * a box reaches outside iff one of its corners is outside (the cube is convex);
//  * a box lies outside (up to a zero-volume touch) iff an axis L separates it from the
//    cube: the box axes e_k, the cube axes u_j and, in 3-D, e_k x u_j (|L|^2 < 1e-20
//    skipped); on L: |L.(b - c)| >= sum_k h_k |L_k| + a sum_j |L.u_j| (b, h: box centre
//    and half edges).
#pragma once

#include <hip/hip_runtime.h>

namespace fcw {

struct CubeGeo {
  int on;         // 0: no cube (the box minus the voids is the physical domain)
  int dim;
  double c[3];
  double a;       // half edge
  double T[9];    // row-major [3][3] (k, j): component k of axis j
};

__host__ __device__ inline bool cube_point_outside(const CubeGeo& g, const double* x) {
#pragma clang fp contract(off)
  for (int j = 0; j < g.dim; ++j) {
    double l = (x[0] - g.c[0]) * g.T[0 * 3 + j];
    for (int k = 1; k < g.dim; ++k) l = l + (x[k] - g.c[k]) * g.T[k * 3 + j];
    if (fabs(l) > g.a) return true;
  }
  return false;
}

// (reaches outside the cube, lies outside it) for the box [lo, hi]
__host__ __device__ inline void cube_box(const CubeGeo& g, const double* lo, const double* hi,
                                         bool& reach, bool& outside) {
#pragma clang fp contract(off)
  reach = false;
  const int nc = 1 << g.dim;
  for (int m = 0; m < nc && !reach; ++m) {
    // corner m: bit k picks lo / hi along k, the same corners as the lexicographic
    // (0/1 per direction) enumeration
    double x[3];
    for (int k = 0; k < g.dim; ++k) x[k] = ((m >> (g.dim - 1 - k)) & 1) ? hi[k] : lo[k];
    reach = cube_point_outside(g, x);
  }
  outside = false;
  const int naxes = (g.dim == 3) ? 15 : 4;
  for (int q = 0; q < naxes && !outside; ++q) {
    double L[3] = {0.0, 0.0, 0.0};
    if (q < g.dim) {
      L[q] = 1.0;
    } else if (q < 2 * g.dim) {
      const int j = q - g.dim;
      for (int k = 0; k < g.dim; ++k) L[k] = g.T[k * 3 + j];
    } else {
      const int k = (q - 6) / 3, j = (q - 6) % 3;
      const double u0 = g.T[0 * 3 + j], u1 = g.T[1 * 3 + j], u2 = g.T[2 * 3 + j];
      if (k == 0) { L[0] = 0.0; L[1] = -u2; L[2] = u1; }
      else if (k == 1) { L[0] = u2; L[1] = 0.0; L[2] = -u0; }
      else { L[0] = -u1; L[1] = u0; L[2] = 0.0; }
      if ((L[0] * L[0] + L[1] * L[1]) + L[2] * L[2] < 1e-20) continue;
    }
    double dist = (0.5 * (lo[0] + hi[0]) - g.c[0]) * L[0];
    double ra = (0.5 * (hi[0] - lo[0])) * fabs(L[0]);
    for (int k = 1; k < g.dim; ++k) {
      dist = dist + (0.5 * (lo[k] + hi[k]) - g.c[k]) * L[k];
      ra = ra + (0.5 * (hi[k] - lo[k])) * fabs(L[k]);
    }
    double rb = 0.0;
    for (int j = 0; j < g.dim; ++j) {
      double proj = g.T[0 * 3 + j] * L[0];
      for (int k = 1; k < g.dim; ++k) proj = proj + g.T[k * 3 + j] * L[k];
      rb = rb + fabs(proj);
    }
    outside = fabs(dist) >= ra + g.a * rb;
  }
}

}  // namespace fcw
