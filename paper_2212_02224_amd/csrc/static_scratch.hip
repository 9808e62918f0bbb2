// static_scratch.hip -- working memory of plan_lower_solve_static in a
// file-scope device array, so that call allocates nothing.
//
// The array is a module global: every GPU the library runs on holds its own
// copy (at its own address) from the first use of the code object until the
// process ends. Host code never passes the array's name to a kernel or a
// copy; it passes the device address that hipGetSymbolAddress returned for
// the current device, taken once per device at plan_create.
//
// Layout (each part 256-byte aligned):
//   [0, kStaticDescBytes)            one request descriptor (ReqDesc)
//   [kStaticActOff, +256)            act_slots (1) and blk_prefix (up to 9)
//   [kStaticZsOff, +kStaticRows*kZ*4) free-coefficient rows of the samples
// Every call rewrites the descriptor and the launch arrays before its
// kernels run, and the kernels write each zs row before anything reads it,
// so nothing needs clearing between calls. Calls that overlap on one GPU
// (two host threads, or two handles on different streams) share the array
// and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan_internal.h"

namespace plan {

namespace {

constexpr size_t kAlign = 256;
constexpr size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kStaticDescBytes = round_up(sizeof(ReqDesc));
constexpr size_t kStaticActOff = kStaticDescBytes;
constexpr size_t kStaticZsOff = kStaticActOff + kAlign;
constexpr size_t kStaticBytes = kStaticZsOff + round_up((size_t)kStaticRows * kZ * sizeof(float));
static_assert(sizeof(int32_t) * (1 + 9) <= kAlign, "launch arrays must fit their part");

// The scratch array itself (about 260 KB).
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kStaticBytes; }

hipError_t static_scratch_init(int device, StaticScratch *out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_addr[device] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_addr[device] = ptr;
  }
  unsigned char *base = static_cast<unsigned char *>(g_addr[device]);
  out->desc = reinterpret_cast<ReqDesc *>(base);
  out->act = reinterpret_cast<int32_t *>(base + kStaticActOff);
  out->zs = reinterpret_cast<float *>(base + kStaticZsOff);
  out->rows = kStaticRows;
  return hipSuccess;
}

}  // namespace plan
