// dh_conservation_noalloc: the FP64 conservation sums of dh_conservation on caller device
// buffers, for callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  The block partials of the
// reduction live in a file-scope device array instead of a handle's buffers; the call
// allocates nothing, synchronises nothing and writes its results to device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/diffhydro.h"
#include "dh_kernels.h"

namespace {

// block partials of one sample: 8 sums x dh::sum_blocks(n^3) blocks; n <= 256 needs 8192
// blocks, 512 KiB per device (held from the first call on a device until the process ends)
constexpr int kMaxN = 256;
constexpr long long kScratchDoubles = 8LL * 8192;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// out[5..7] *= m_dm (the dark-matter momentum sums as mass times p)
__global__ void scale_dm_kernel(double* out, double m_dm) {
  const int k = threadIdx.x;
  if (k < 3) out[5 + k] *= m_dm;
}

// The device address of `scratch` on the current device, looked up once per device.
int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(DH_E_HIP, "dh_conservation_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DH_E_HIP, std::string("dh_conservation_noalloc: hipGetSymbolAddress: ") +
                                hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return DH_OK;
}

}  // namespace

const char* dh_noalloc_last_error_message() { return g_err.c_str(); }

extern "C" {

int dh_conservation_noalloc(const float* d_q, const float* d_mom, int32_t n, int32_t batch,
                            double m_dm, double* d_out, void* hip_stream) {
  g_err.clear();
  if (!d_q || !d_mom || !d_out) return fail(DH_E_INVAL, "dh_conservation_noalloc: null pointer");
  if (n < 1 || batch < 1) return fail(DH_E_INVAL, "dh_conservation_noalloc: n and batch must be >= 1");
  if (n > kMaxN)
    return fail(DH_E_INVAL, "dh_conservation_noalloc: n = " + std::to_string(n) +
                                " exceeds the scratch limit n <= " + std::to_string(kMaxN));
  const long long nc = static_cast<long long>(n) * n * n;
  const int nb = dh::sum_blocks(nc);
  if (8LL * nb > kScratchDoubles)
    return fail(DH_E_INVAL, "dh_conservation_noalloc: partials exceed the scratch array");
  double* part = nullptr;
  if (const int rc = scratch_on_current_device(&part)) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    // samples one after another on the stream, each over the whole scratch (stream order
    // keeps a sample's partials until its reduction has read them)
    for (int i = 0; i < batch; ++i) {
      double* out = d_out + 8LL * i;
      dh::launch_conservation_partial(st, d_q + 5 * nc * i, d_mom + 3 * nc * i, part, nb, nc);
      dh::launch_reduce_sum(st, part, nb, nb, 8, out);
      hipLaunchKernelGGL(scale_dm_kernel, dim3(1), dim3(64), 0, st, out, m_dm);
      DH_LAUNCH_CHECK();
    }
  } catch (const std::exception& e) {
    return fail(DH_E_HIP, e.what());
  }
  return DH_OK;
}

}  // extern "C"
