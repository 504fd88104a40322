// Definitions shared by the step kernels (generic tile kernel and the 2-D kernel).
#pragma once

#include <cmath>

#include "common.h"

namespace fcw {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
  const T* ycut;  // [nrhs][ncand][n_loc] cut-cell products of this step (step / apply)
  const void* kref_bf;  // [n_loc^2] bf16 K_ref (BF16 form)
  int64_t ncand;
  // Batched launches (several problems of one kind; step mode only): the launch argument
  // carries nprob > 0, the device records of the problems and the first block of each
  // (bstart[nprob] = grid size), and the step index jstep of the call.  A record holds
  // the caller's state in u_out and its ping-pong partner in u_alt, the time origin t0,
  // the step dt, the step count and right-hand sides of its call, and start as for the
  // whole call; the kernel derives u_in / u_out, t and start of step jstep from them.
  const StepArgs* probs;
  const int32_t* bstart;
  int nprob, jstep;
  T* u_alt;
  double t0, dt;
  int nsteps, nrhs;
};

// Workgroup barrier of the step kernels: this wave's LDS operations are complete
// (lgkmcnt(0)) and every wave has arrived.  Unlike __syncthreads() it does not also wait
// for outstanding vector-memory operations (its release fence does): the step kernels
// keep loads for later rows or layers, and their stores, in flight across barriers and
// order them with explicit vmcnt waits.  No step kernel reads global data written by
// another wave of the same launch.
__device__ static inline void block_sync() {
  asm volatile("" ::: "memory");
  // lgkmcnt(0); vmcnt (63) and expcnt (7) not waited for
  __builtin_amdgcn_s_waitcnt((15 & 15) | (7 << 4) | (0 << 8) | (3 << 14));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__device__ static inline double ricker(double t, double f0) {
  const double pi = 3.14159265358979323846;
  const double ts = 2.0 * sqrt(6.0) / (pi * f0);
  const double q = pi * f0 * (t - ts);
  return (1.0 - 2.0 * q * q) * exp(-q * q);
}

}  // namespace fcw
