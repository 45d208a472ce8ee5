// bse_spectrum_noalloc: bse_spectrum for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  Its partial
// results (the oscillator strength of each exciton) live in a file-scope
// device array instead of a caller workspace; every GPU the library runs on
// holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bse.h"
#include "kernels.h"

namespace {

constexpr int kMaxDevices = 64;

// One double per exciton: |t_l|^2 averaged over the polarisations.
static __device__ __align__(256) double scratch[BSE_NOALLOC_MAX_NLAM];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // address of `scratch` on each device, once looked up

// The device address of this device's copy of `scratch`: looked up once per
// device, with that device current (the array's host-side name is not a
// device address).
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_ptr[dev]);
  return hipSuccess;
}

}  // namespace

// Error reporting and argument checks shared with bse_spectrum (bse_api.cpp).
namespace bse {
int api_fail(int code, const char* msg);
int api_spectrum_args(int ns, int nlam, const double* E, const double* A, const double* d, int nq, int nk,
                      double omega_cell, int nw, double eta_eV, double* eps2);
}  // namespace bse

extern "C" int bse_spectrum_noalloc(int ns, int nlam, const double* E, const double* A, const double* d, int nq,
                                    int nk, double omega_cell, int nw, double w0_eV, double w1_eV, double eta_eV,
                                    double* eps2, void* stream) {
  int rc = bse::api_spectrum_args(ns, nlam, E, A, d, nq, nk, omega_cell, nw, eta_eV, eps2);
  if (rc) return rc;
  if (nlam > BSE_NOALLOC_MAX_NLAM)
    return bse::api_fail(BSE_ERR_WORKSPACE, "nlam above BSE_NOALLOC_MAX_NLAM: the static scratch holds that many excitons");
  // k_spec_t writes every one of the nlam entries that k_spec_eps2 then
  // reads, so the array needs no clearing between calls
  double* t2 = nullptr;
  hipError_t e = scratch_ptr(&t2);
  if (e != hipSuccess) return bse::api_fail(BSE_ERR_HIP, hipGetErrorString(e));
  e = bse::launch_spectrum(ns, nlam, nq, E, reinterpret_cast<const double2*>(A), reinterpret_cast<const double2*>(d),
                           (double)nk * omega_cell, nw, w0_eV, w1_eV, eta_eV, t2, eps2,
                           reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return bse::api_fail(BSE_ERR_HIP, hipGetErrorString(e));
  return BSE_OK;
}
