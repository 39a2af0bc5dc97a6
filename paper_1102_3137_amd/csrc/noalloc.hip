// Allocation-free entry point: the whole hot path of dyson_solve with its
// workspace carved out of one file-scope device array instead of allocated,
// for callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid it).
//
// Each device that the library runs on holds one copy of the array (kScratch
// bytes) from the first dyson_create on it until the process ends.  Every
// dyson_solve_noalloc call on a device uses that device's copy and leaves its
// contents behind: calls that overlap on one device (from several threads,
// or on several streams) race on it and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/dyson.h"
#include "engine.h"

namespace {

// 256 MiB: room for a full-rank solve of, e.g., a 64^2 lattice over 16
// frequencies or a 96^2 lattice over 4 (dyson_noalloc_bytes gives the exact need).
constexpr size_t kScratch = size_t(256) << 20;

static __device__ __align__(256) unsigned char scratch[kScratch];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

namespace dyson {

// The array's name in host code is only a host-side stand-in: its device
// address differs per device and comes from the runtime, once per device,
// with that device current.
dyson_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device ordinal beyond the scratch table");
    return DYSON_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_mu);
  if (g_addr[device]) return DYSON_OK;
  if (hipSetDevice(device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return DYSON_EDEVICE;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    return DYSON_EDEVICE;
  }
  g_addr[device] = ptr;
  return DYSON_OK;
}

}  // namespace dyson

extern "C" {

size_t dyson_noalloc_max_bytes(void) { return kScratch; }

dyson_status dyson_noalloc_bytes(const dyson_plan* p, int K, size_t* bytes) {
  if (!p || !bytes || K < 1) {
    dyson::set_error("bad argument");
    return DYSON_EINVAL;
  }
  *bytes = dyson::carved_bytes(p, K);
  return DYSON_OK;
}

dyson_status dyson_solve_noalloc(dyson_plan* p, int K, const double* d_V, const double* d_omega,
                                 const double* d_sigma, double* d_G, void* stream,
                                 dyson_report* report) {
  using namespace dyson;
  if (!p || !p->ctx) {
    set_error("plan has no device context");
    return DYSON_EINVAL;
  }
  if (K < 1 || K > 65535) {
    set_error("K must be in [1, 65535]");
    return DYSON_EINVAL;
  }
  const int dev = p->ctx->device;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = (dev >= 0 && dev < kMaxDevices) ? g_addr[dev] : nullptr;
  }
  if (!base) {  // dyson_create records it; nothing is allocated here
    set_error("the device's scratch array was not set up (dyson_create)");
    return DYSON_EDEVICE;
  }
  if (hipSetDevice(dev) != hipSuccess) {
    set_error("hipSetDevice failed");
    return DYSON_EDEVICE;
  }
  hipStream_t s = (hipStream_t)stream;
  dyson_status st = carve_work(p, &p->carved, K, (char*)base, kScratch);
  if (st != DYSON_OK) return st;
  Slice sl{K, d_V, d_omega, d_sigma, d_G, 0};
  st = validate_slices(p, &p->carved, &sl, 1, s);
  if (st != DYSON_OK) return st;
  return run_solve(p, &p->carved, &sl, 1, s, report, nullptr);
}

}  // extern "C"
