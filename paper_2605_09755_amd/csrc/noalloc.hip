// Allocation-free form of the sketch pass At = A S (rf_sketch_apply_noalloc).
//
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid allocation): the sketch table, its
// kernel-ready form and the per-chunk bucket occupancy live in one file-scope
// device array, `scratch`, instead of a caller workspace.  Each GPU the library
// runs on holds its own copy of the array until the process ends.  Host code
// never passes the array's name to a kernel (in host code it is only a stand-in
// symbol); it looks up the array's device address once per device with
// hipGetSymbolAddress and passes that address.
//
// Every call on a GPU shares that GPU's array and leaves its contents behind;
// nothing in it has to start at zero (every word a call reads was written
// earlier in the same call).  Calls that overlap on one GPU (two streams, two
// threads) race on the array.
#include <mutex>

#include "../../include/rf.h"
#include "common.h"
#include "kernels.h"

using namespace rf;

constexpr size_t kScratchBytes = (size_t)8 << 20;  // 8 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, set on first use

// Device address of this device's `scratch` (looked up once per device, with the
// device current).
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of `scratch` one call needs: sketch table, ready table, chunk occupancy or
// the gather form's bucket lists.
size_t noalloc_bytes(int64_t n, int s, int r1) {
  return round256((size_t)n * s * sizeof(int32_t)) + round256((size_t)n * s * sizeof(uint32_t)) +
         round256(sketch_right_work_ints(n, s, r1) * sizeof(int));
}

}  // namespace

extern "C" {

rf_status rf_sketch_apply_noalloc(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo, void* stream) {
  if (!A || !A->data || A->rows < 1 || A->cols < 1 || A->ld < A->cols || A->reserved != 0) return RF_EINVAL;
  if (A->dtype != RF_F32 && A->dtype != RF_BF16 && A->dtype != RF_FP8E4M3_B128) return RF_EINVAL;
  if ((A->dtype == RF_FP8E4M3_B128) != (A->block_scales != nullptr)) return RF_EINVAL;
  if (!p || p->sketch < 1 || p->nnz_per_col < 1 || p->nnz_per_col > p->sketch || !out || ldo < p->sketch)
    return RF_EINVAL;
  const int64_t m = A->rows, n = A->cols;
  const int s = p->nnz_per_col, r1 = p->sketch;
  if (noalloc_bytes(n, s, r1) > kScratchBytes) return RF_EUNSUPPORTED;
  void* base = nullptr;
  if (scratch_address(&base) != hipSuccess) return RF_EHIP;
  unsigned char* q = static_cast<unsigned char*>(base);
  int32_t* table = reinterpret_cast<int32_t*>(q);
  q += round256((size_t)n * s * sizeof(int32_t));
  uint32_t* ready = reinterpret_cast<uint32_t*>(q);
  q += round256((size_t)n * s * sizeof(uint32_t));
  int* cmax = reinterpret_cast<int*>(q);
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_sketch_table(n, s, r1, p->seed, 0, 0, table, st);
  const bool fast = sketch_right_fast_ok(s) && !sketch_right_gather(s, n, r1);
  if (e == hipSuccess && fast) e = launch_sketch_ready(table, n, s, r1, sketch_right_cpl(s), ready, st);
  if (e == hipSuccess)
    e = launch_sketch_right(A->dtype, A->data, A->ld, A->block_scales, table, fast ? ready : nullptr, cmax, s, m, n,
                            r1, out, ldo, st);
  return e == hipSuccess ? RF_OK : RF_EHIP;
}

}  // extern "C"
