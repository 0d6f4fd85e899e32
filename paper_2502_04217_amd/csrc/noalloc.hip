// Training-loss gradient of the learned correction for callers that cannot
// allocate device memory (code under HIP graph capture, tight loops, hosts
// that forbid allocation): csipm_mlp_loss_grad_noalloc runs the kernels of
// csipm_mlp_loss_grad with their per-workgroup gradient partials in a fixed
// device array of this file instead of a caller workspace.
//
// The array holds the partials of at most CSIPM_MLP_NOALLOC_MAX_REC records
// (one row of 1249 gradient sums and the loss per MLP_REC_PER_BLOCK
// records, 9.8 MiB); every GPU the library runs on keeps its own copy until
// the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// passed to kernels.  Each workgroup writes its whole row before the reduce
// kernel reads it, so nothing has to be cleared between calls; calls that
// overlap on one GPU (other streams, other host threads) share the array
// and race.
#include "../../include/csipm.h"

#include <mutex>
#include <string>

#include "mlp.h"

constexpr int kNoallocRows = (CSIPM_MLP_NOALLOC_MAX_REC + csipm::MLP_REC_PER_BLOCK - 1) / csipm::MLP_REC_PER_BLOCK;
constexpr size_t kNoallocRowDoubles = (size_t)csipm::MLP_NP + 1;
static_assert(kNoallocRows * kNoallocRowDoubles * sizeof(double) < (size_t)16 << 20, "the fixed scratch stays modest");

// the gradient partials of one call: row b = workgroup b (1249 sums, loss)
static __device__ __align__(256) double scratch[kNoallocRows * kNoallocRowDoubles];

namespace csipm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[dev] = static_cast<double*>(p);
  }
  *out = g_addr[dev];
  return hipSuccess;
}

thread_local std::string g_err;

csipm_status fail(csipm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

}  // namespace

const char* noctx_last_error() { return g_err.c_str(); }
void noctx_set_error(const std::string& msg) { g_err = msg; }

}  // namespace csipm

extern "C" csipm_status csipm_mlp_loss_grad_noalloc(const float* d_params, const float* d_feat, const float* d_rec,
                                                    int n_rec, double* d_loss_out, float* d_grad, void* hip_stream) {
  using namespace csipm;
  if (!d_params || !d_feat || !d_rec || !d_loss_out || !d_grad || n_rec < 1)
    return fail(CSIPM_EINVAL, "mlp_loss_grad_noalloc: null pointer or n_rec < 1");
  if (n_rec > CSIPM_MLP_NOALLOC_MAX_REC)
    return fail(CSIPM_ENOMEM, "mlp_loss_grad_noalloc: n_rec = " + std::to_string(n_rec) +
                                  " exceeds the fixed scratch (at most " +
                                  std::to_string(CSIPM_MLP_NOALLOC_MAX_REC) +
                                  " records); use csipm_mlp_loss_grad with a workspace");
  double* sc = nullptr;
  hipError_t e = scratch_address(&sc);
  if (e != hipSuccess)
    return fail(CSIPM_EHIP, std::string("mlp_loss_grad_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
  mlp_loss_grad(d_params, d_feat, d_rec, n_rec, d_loss_out, d_grad, sc, reinterpret_cast<hipStream_t>(hip_stream));
  e = hipGetLastError();
  if (e != hipSuccess) return fail(CSIPM_EHIP, std::string("mlp_loss_grad_noalloc: ") + hipGetErrorString(e));
  return CSIPM_OK;
}
