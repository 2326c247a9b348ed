// Dense eigen-decomposition without any device allocation: the same batched
// Jacobi kernels as iesh_eigh_batched, with the work space of orders above
// the LDS limit taken from a fixed array in device memory instead of from
// hipMalloc.
//
// The array `scratch` is a file-scope __device__ array; every GPU the library
// runs on holds its own copy until the process ends.  Host code must not pass
// its name to a kernel (on the host it is only a stand-in symbol): the device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept in g_scratch_ptr.  Every call on a device shares
// that device's array, so calls that overlap on one GPU (different streams,
// or different host threads) race; calls on one stream are ordered by it.
// The Jacobi kernel initialises every work-space element it reads (the
// matrix from H, the rotations from the identity), so nothing needs to be
// cleared between calls.

#include <mutex>
#include <string>

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr size_t kScratchDoubles = (size_t)IESH_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace
}  // namespace iesh

extern "C" int iesh_eigh_batched_noalloc(const double* H, int32_t n, int32_t batch, double* lam,
                                         double* Q, int32_t* sweeps, void* hip_stream) {
  using namespace iesh;
  set_call_error("");
  if (n < 1 || n > IESH_JACOBI_MAX_N) {
    set_call_error("eigh_noalloc: n out of range [1, IESH_JACOBI_MAX_N]");
    return IESH_EINVAL;
  }
  if (batch < 0) {
    set_call_error("eigh_noalloc: batch must be >= 0");
    return IESH_EINVAL;
  }
  const size_t need = jacobi_work_elems(n, batch);
  if (need > kScratchDoubles) {
    set_call_error("eigh_noalloc: batch x work space (" + std::to_string(need * sizeof(double)) +
                   " bytes) exceeds the fixed scratch of " +
                   std::to_string((size_t)IESH_NOALLOC_SCRATCH_BYTES) + " bytes; split the batch");
    return IESH_EINVAL;
  }
  if (batch == 0) return IESH_OK;
  if (!H || !lam || !Q) {
    set_call_error("eigh_noalloc: H, lam and Q must be given");
    return IESH_EINVAL;
  }
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e == hipSuccess && (device < 0 || device >= kMaxDevices)) e = hipErrorInvalidDevice;
  double* work = nullptr;
  if (e == hipSuccess && need) e = scratch_address(device, &work);
  if (e == hipSuccess)
    e = launch_jacobi(H, n, batch, lam, Q, sweeps, work, reinterpret_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    set_call_error(std::string("eigh_noalloc: ") + hipGetErrorString(e));
    return IESH_EDEVICE;
  }
  return IESH_OK;
}
