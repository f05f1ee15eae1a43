// Prefactored solve with its working memory in a fixed device array, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc). The solve and its kernels
// are the ones of qnsim_solve_device; only the buffers differ: the permuted
// right-hand side, the forward intermediate, the children's update layers,
// the dense top block's partial products and the permuted solution are carved
// out of `scratch`, a file-scope device array of kNoAllocBytes that every
// device the library runs on holds until the process ends.
//
// In host code the name `scratch` is a host-side stand-in, not a device
// address. The device address is looked up once per device, with that device
// current, by hipGetSymbolAddress, and only that pointer is handed to
// kernels. All calls on one device share the array and it keeps the last
// call's contents: the update layers, which the solve needs zero wherever no
// child writes, are cleared by a fill kernel in every call. Calls that
// overlap on one device (two streams, two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qnsim.h"
#include "kernels.hpp"

namespace qn {

namespace {

constexpr size_t kNoAllocBytes = size_t(16) << 20;           // 16 MiB per device
constexpr size_t kNoAllocDoubles = kNoAllocBytes / sizeof(double);
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kNoAllocDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device

__global__ void __launch_bounds__(256) k_fill_zero(double* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Doubles rounded up to whole 256-byte lines.
inline size_t lines(size_t doubles) { return (doubles + 31) / 32 * 32; }

}  // namespace

int dev_solve_noalloc(DeviceMesh& D, const double* q, double* r, void* stream, std::string& err) {
  if (D.device < 0 || D.device >= kMaxDevices) {
    err = "device ordinal out of range for the fixed scratch array";
    return QNSIM_E_INVALID;
  }
  const size_t v3 = lines(3 * (size_t)D.nf);
  const size_t vp = lines((size_t)D.vp_len);
  const size_t tt = lines(D.top_n > 0 ? top_part_doubles(D.top_n) : 0);
  const size_t need = 3 * v3 + vp + tt;  // q, z, r; update layers; top partial products
  if (need > kNoAllocDoubles) {
    err = "the solve needs " + std::to_string(need * sizeof(double)) +
          " bytes of working memory; the fixed scratch array holds " +
          std::to_string(kNoAllocBytes);
    return QNSIM_E_INVALID;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) {
    err = "hipGetDevice failed";
    return QNSIM_E_DEVICE;
  }
  if (cur != D.device && hipSetDevice(D.device) != hipSuccess) {
    err = "hipSetDevice failed";
    return QNSIM_E_DEVICE;
  }
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[D.device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        if (cur != D.device) (void)hipSetDevice(cur);
        err = std::string("hipGetSymbolAddress of the scratch array failed: ") +
              hipGetErrorString(e);
        return QNSIM_E_DEVICE;
      }
      g_ptr[D.device] = static_cast<double*>(p);
    }
    base = g_ptr[D.device];
  }
  hipStream_t st = (hipStream_t)stream;
  double* qs = base;
  double* zs = qs + v3;
  double* rs = zs + v3;
  double* vps = rs + v3;
  double* top = vps + vp;
  const long long nvp = (long long)D.vp_len;
  if (nvp > 0)
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nvp + 255) / 256)), dim3(256), 0, st, vps,
                       nvp);
  launch_load_perm(st, D.nf, D.vperm, q, qs);
  const SolveScratch scr{zs, vps, top};
  launch_solve(D, st, qs, rs, nullptr, nullptr, &scr);
  launch_store_perm(st, D.n, D.nf, D.vperm, rs, r);
  const hipError_t e = hipGetLastError();
  if (cur != D.device) (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    err = std::string("solve launch failed: ") + hipGetErrorString(e);
    return QNSIM_E_DEVICE;
  }
  return 0;
}

}  // namespace qn
