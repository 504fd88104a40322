// Allocation-free form of the explicit step (fcw_step_explicit_noalloc in fcw.h).
//
// The step needs three device work areas besides the caller's state and the context's
// matrices: the point-source load vectors, the cut-cell products of the current step and
// the ping-pong partner of u.  fcw_step_explicit allocates them in the context on first
// use; here they live in one fixed device array of FCW_NOALLOC_SCRATCH_BYTES, so the call
// makes no device allocation and can run where the caller cannot allocate.
//
// The array's host-side name is not a device address.  Its address on each device is
// looked up once, with that device current, through hipGetSymbolAddress, and only that
// address is handed to kernels and copies.  Every call on one device shares the array:
// calls that overlap on one device (other threads, other streams) race.  None of the
// three areas needs clearing: each step writes its products and partner state before
// reading them, and the load vectors are staged anew by every call.
#include <mutex>

#include "common.h"

static __device__ __align__(256) unsigned char scratch[FCW_NOALLOC_SCRATCH_BYTES];

namespace fcw {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

fcw_status scratch_address(void** out) {
  int dev = -1;
  FCW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the allocation-free step tracks", dev,
              kMaxDevices);
    return FCW_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    FCW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned a null address for the scratch array");
      return FCW_E_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FCW_OK;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace fcw

using namespace fcw;

extern "C" fcw_status fcw_step_explicit_noalloc(fcw_ctx* c, int32_t nrhs, void* u, void* d,
                                                const fcw_source* src, double t0, double dt,
                                                int32_t nsteps, int32_t start) {
  clear_error();
  fcw_status st = check_step_call(c, nrhs, u, d, src, dt, nsteps);
  if (st) return st;
  const size_t sb = c->state_bytes();
  const size_t src_bytes = align256((size_t)kMaxSrc * (sizeof(SourceDev) + sizeof(fcw_source)));
  const size_t ycut_bytes = (size_t)nrhs * c->n_cut_cand * c->n_loc * sb;
  const size_t ubuf_bytes = (size_t)nrhs * c->ndof * sb;
  const size_t need = src_bytes + align256(ycut_bytes) + align256(ubuf_bytes);
  if (need > (size_t)FCW_NOALLOC_SCRATCH_BYTES) {
    set_error("the allocation-free step needs %zu bytes of scratch for %d right-hand side(s) "
              "of %lld DOFs; it holds %zu (use fcw_step_explicit)",
              need, nrhs, (long long)c->ndof, (size_t)FCW_NOALLOC_SCRATCH_BYTES);
    return FCW_E_ARG;
  }
  if (nsteps == 0) return FCW_OK;
  void* base = nullptr;
  if ((st = scratch_address(&base))) return st;
  char* p = static_cast<char*>(base);

  // Point the context's work areas into the array for this call only; the context's
  // own buffers (and the record of the sources staged in them) come back afterwards.
  SourceDev* own_src = c->d_src;
  void* own_ycut = c->d_ycut;
  const size_t own_ycut_bytes = c->ycut_bytes;
  c->d_src = reinterpret_cast<SourceDev*>(p);
  c->d_ycut = p + src_bytes;
  c->ycut_bytes = ycut_bytes;
  if (src) st = prepare_sources(*c, nrhs, src, /*remember=*/false);
  if (!st) {
    if (!src) c->d_src = nullptr;
    st = run_steps(*c, c->tile_choice, nrhs, u, d, p + src_bytes + align256(ycut_bytes), t0, dt,
                   nsteps, start);
  }
  c->d_src = own_src;
  c->d_ycut = own_ycut;
  c->ycut_bytes = own_ycut_bytes;
  return st;
}
