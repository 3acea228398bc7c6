// sl7_simulate_noalloc: sl7_simulate for callers that cannot allocate device
// memory (code under stream capture, tight serving loops).  Its scratch --
// the instance record, the work-queue counter and order, the 64-path block
// partials and the finalize sums -- lives in one fixed device array of this
// library, so a call allocates nothing.  The kernels are the ones
// sl7_simulate launches; only the place of their scratch differs.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "sl7_host.hpp"

namespace sl7 {

// Scratch layout (byte offsets): instance record, work-order prefix sums and
// order, work-queue counter, statistics (when the caller passes none),
// finalize sums, then one 64-byte partial per 64-path block.
constexpr size_t kStInst = 0;
constexpr size_t kStPrefix = 2048;
constexpr size_t kStOrder = 2304;
constexpr size_t kStCounter = 2560;
constexpr size_t kStStats = 2816;
constexpr size_t kStChunks = 4096;
constexpr size_t kStPartials = 64 * 1024;
constexpr int64_t kStMaxBlocks = (int64_t)1 << 18;  // N <= 2^24 paths
constexpr size_t kStBytes = kStPartials + (size_t)kStMaxBlocks * sizeof(Partial);
static_assert(sizeof(InstDev) <= kStPrefix - kStInst, "instance record slot");
static_assert(sizeof(sl7_stats) <= kStChunks - kStStats, "statistics slot");

// One copy per device (16.06 MiB), held until the process ends.  Host code
// never passes this name to a kernel or copy: it uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStBytes];

// Writes the instance record (a kernel argument) and the one-instance work
// order into the scratch, and zeroes the work-queue counter.
__global__ __launch_bounds__(64) void k_static_setup(InstDev I, InstDev* dst, int64_t* prefix,
                                                     int32_t* order, unsigned long long* counter,
                                                     int64_t n_items) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(&I);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(InstDev) / 4); i += blockDim.x) d[i] = s[i];
  if (threadIdx.x == 0) {
    prefix[0] = 0;
    prefix[1] = n_items;
    order[0] = 0;
    counter[0] = 0;
  }
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
unsigned char* g_static_ptr[kMaxDevices];
int g_static_ncu[kMaxDevices];

// The scratch's address on device `dev` (current), looked up once per device.
int static_scratch(int dev, unsigned char** ptr, int* n_cu) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SL7_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)");
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CU count)");
    g_static_ncu[dev] = ncu > 0 ? ncu : 256;
    g_static_ptr[dev] = (unsigned char*)p;
  }
  *ptr = g_static_ptr[dev];
  *n_cu = g_static_ncu[dev];
  return SL7_OK;
}

}  // namespace
}  // namespace sl7

using namespace sl7;

extern "C" int sl7_simulate_noalloc(const sl7_problem* pr, const sl7_mlp* Hc, int prec,
                                    uint64_t seed, void* YT_dev, sl7_stats* stats_dev,
                                    const sl7_plan* plan_in, void* stream) {
  const Mlp* H = reinterpret_cast<const Mlp*>(Hc);
  int rc = check_problem(pr, H, prec, "pr");
  if (rc) return rc;
  if (is_pwl(prec))
    return fail(SL7_EUNSUPPORTED, "sl7_simulate_noalloc: the piecewise-linear modes build "
                                  "per-instance tables (use sl7_simulate)");
  const int64_t blocks = (pr->N + 63) / 64;
  if (blocks > kStMaxBlocks)
    return fail(SL7_EINVAL, "sl7_simulate_noalloc: pr.N=%lld exceeds the fixed scratch "
                            "(at most %lld paths)", (long long)pr->N,
                (long long)(kStMaxBlocks * 64));
  int dev;
  rc = current_device(&dev);
  if (rc) return rc;
  unsigned char* base;
  int n_cu;
  rc = static_scratch(dev, &base, &n_cu);
  if (rc) return rc;
  sl7_plan plan;
  if (plan_in) plan = *plan_in; else default_plan(prec, blocks, n_cu, &plan);
  rc = check_plan(&plan, prec);
  if (rc) return rc;
  if (H) {
    // the network's device copy must exist already: creating it allocates
    const bool resident = H->device == dev &&
                          (prec == SL7_F64 ? (H->lane64 != nullptr) : (H->pack[prec] != nullptr));
    if (!resident)
      return fail(SL7_EINVAL, "sl7_simulate_noalloc: H has no device copy for prec %d on device "
                              "%d (one sl7_simulate or sl7_eval_H call with it makes one)",
                  prec, dev);
  }
  SimArgs a;
  std::memset(&a, 0, sizeof(a));
  double x[SL7_MAX_M];
  rc = fill_nodes(pr->m, a, x);
  if (rc) return rc;
  InstDev I;
  fill_inst(*pr, H, x, I);
  I.part_offset = 0;
  I.yt_offset = 0;
  InstDev* inst = (InstDev*)(base + kStInst);
  int64_t* prefix = (int64_t*)(base + kStPrefix);
  int32_t* order = (int32_t*)(base + kStOrder);
  unsigned long long* counter = (unsigned long long*)(base + kStCounter);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(64), 0, s, I, inst, prefix, order, counter,
                     blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch static setup");
  a.inst = inst;
  a.item_prefix = prefix;
  a.order = order;
  a.n_order = 1;
  a.n_items = blocks;
  a.counter = counter;
  a.partials = (Partial*)(base + kStPartials);
  a.YT = YT_dev;
  a.seed = seed;
  sl7_stats* stats = stats_dev ? stats_dev : (sl7_stats*)(base + kStStats);
  return launch_sequence(a, 1, pr->N, H, prec, plan, s, n_cu, base + kStChunks, stats);
}
