// aaq_energy_grad_noalloc: the energy + adjoint gradient entry point for callers that cannot
// allocate device memory.  Its workspace (the instance block, phase tables, per-sweep
// scales and per-tile partial sums of aaq_energy_grad) is a static device array of
// AAQ_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "aaq_launch.h"
#include "aaqaoa.h"

namespace {

// In host code this name is a host-side stand-in, not a device address: kernels get the
// address that hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) unsigned char scratch[AAQ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device, looked up once per device with
// that device current
aaq_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return aaq::set_error(AAQ_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return aaq::set_error(AAQ_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return aaq::set_error(AAQ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return AAQ_OK;
}

}  // namespace

extern "C" aaq_status aaq_energy_grad_noalloc(const aaq_problem* prob, int p, const double* gamma,
                                              const double* beta, aaq_observable obs, aaq_precision prec,
                                              void* d_state, size_t state_bytes, void* d_lambda, size_t lambda_bytes,
                                              void* stream, double* energy_out, double* dgamma_out,
                                              double* dbeta_out, double* norm_out) {
  if (!energy_out || !dgamma_out || !dbeta_out) return aaq::set_error(AAQ_ERR_INVALID_ARG, "output pointer is NULL");
  aaq_status s = aaq::validate_call(prob, p, gamma, beta);
  if (s) return s;
  // the workspace bound of aaq_energy_grad (any tile size and state mode), on the host
  size_t need = 0;
  if ((s = aaq_workspace_size(prob, p, 1, obs, AAQ_AGG_FUSED, prec, &need))) return s;
  if (need > AAQ_NOALLOC_SCRATCH_BYTES)
    return aaq::set_error(AAQ_ERR_BUFFER, "the evaluation needs " + std::to_string(need) +
                                              " bytes of workspace; the static scratch holds " +
                                              std::to_string((size_t)AAQ_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  if ((s = scratch_address(&ws))) return s;
  return aaq::energy_grad_pageable(prob, p, gamma, beta, obs, prec, d_state, state_bytes, d_lambda, lambda_bytes, ws,
                                   AAQ_NOALLOC_SCRATCH_BYTES, stream, energy_out, dgamma_out, dbeta_out, norm_out);
}
