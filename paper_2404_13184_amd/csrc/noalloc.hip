// tanq_sample_noalloc: all-qubit sampling that allocates nothing, for callers that cannot call
// hipMalloc (work under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The CDF and the outcomes live in `scratch`, a fixed device array of the library: one copy per
// GPU, resident until the process ends.  Host code never passes the array's name to a kernel or a
// copy (in host code that name is only a host-side stand-in); it looks up the array's device
// address once per device with hipGetSymbolAddress, with that device current, and uses that
// address from then on.
//
// Every call on one GPU shares that GPU's array and leaves its contents behind.  Nothing in it
// has to start at zero: each call's CDF kernel writes all 2^n CDF entries and its draw kernel
// all `shots` outcomes before anything reads them, in stream order.  Calls that overlap on one
// GPU (other threads, or other streams not yet drained) race for the array.
#include <mutex>

#include "abi_util.hpp"

namespace {

constexpr int kNoAllocMaxQubits = 17;              // CDF of up to 2^17 outcomes (1 MiB)
constexpr uint64_t kNoAllocMaxShots = 1ull << 17;  // outcomes per call (1 MiB)
constexpr uint64_t kCdfWords = 1ull << kNoAllocMaxQubits;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint64_t scratch[kCdfWords + kNoAllocMaxShots];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up on the first call there.
void* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) tanq::fail(TANQ_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    int prev = -1;
    TANQ_HIP(hipGetDevice(&prev));
    if (prev != device) TANQ_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) tanq::fail(TANQ_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (!ptr) tanq::fail(TANQ_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

}  // namespace

extern "C" tanq_status tanq_sample_noalloc(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01,
                                           const double* p10, uint64_t* host_out) {
  return tanq::guarded([&] {
    int n = 0, device = 0;
    tanq::sample_check(d, shots, seed, p01, p10, host_out, &n, &device);
    if (n > kNoAllocMaxQubits)
      tanq::fail(TANQ_E_ARG, "tanq_sample_noalloc holds the CDF of at most 2^" + std::to_string(kNoAllocMaxQubits) +
                                 " outcomes; the state has " + std::to_string(n) + " qubits");
    if (shots > kNoAllocMaxShots)
      tanq::fail(TANQ_E_ARG, "tanq_sample_noalloc draws at most " + std::to_string(kNoAllocMaxShots) +
                                 " shots per call; asked for " + std::to_string(shots));
    if (shots == 0) return;
    uint64_t* base = static_cast<uint64_t*>(scratch_on(device));
    tanq::sample_run(d, shots, seed, p01, p10, reinterpret_cast<double*>(base), base + kCdfWords, host_out);
  });
}
