// molt_noalloc.hip -- mol_t_helmholtz_sweep_noalloc: the line inverse of
// mol_t_helmholtz_sweep for callers that cannot allocate device memory.
//
// The y-direction sweep needs scratch memory for its segment totals / seeds
// and the periodic closing-cell quadratures.  Here it lives in one
// file-scope device array, `scratch`, of kScratchBytes, which every device the
// library runs on holds until the process ends.  Its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) and kept;
// kernels are given that address, never the host-side name of the array.
//
// Every call on one device shares that device's array: calls that overlap on
// one device (two streams, two threads) race.  The sweep writes every scratch
// word it later reads, so no clearing is needed between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "molt_internal.h"

namespace molt {
int32_t set_error(int32_t code, const char* msg);
int32_t sweep_check(const molt_grid* g, int32_t axis, double alpha, int32_t precision, const void* d_in,
                    const void* d_out, int64_t batch);
void sweep_scratch_layout(const molt_grid* g, int32_t precision, int64_t batch, size_t* tot_bytes,
                          size_t* jln_bytes);
int32_t sweep_impl(const molt_grid* g, int32_t axis, double alpha, int32_t precision, const void* d_in, void* d_out,
                   int64_t batch, void* tot, void* jln, void* cpy, hipStream_t s);
}  // namespace molt

namespace {
constexpr size_t kScratchBytes = (size_t)MOLT_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "the scratch size is a multiple of 256 bytes");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (nullptr: not looked up yet)

// the current device's address of `scratch` (looked up on the first call on it)
int32_t scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return molt::set_error(MOLT_EHIP, "mol_t_helmholtz_sweep_noalloc: no current HIP device (or more than 64)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return molt::set_error(MOLT_EHIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MOLT_OK;
}
}  // namespace

extern "C" {

size_t molt_noalloc_scratch_bytes(void) { return kScratchBytes; }

int32_t mol_t_helmholtz_sweep_noalloc(const molt_grid* g, int32_t axis, double alpha, int32_t precision,
                                      const void* d_in, void* d_out, int64_t batch, void* stream) {
  molt::set_error(MOLT_OK, "");
  int32_t rc = molt::sweep_check(g, axis, alpha, precision, d_in, d_out, batch);
  if (rc != MOLT_OK) return rc;
  void* tot = nullptr;
  void* jln = nullptr;
  if (axis == 1 && g->ny > 1) {
    if (d_in == d_out)
      return molt::set_error(MOLT_EINVAL, "mol_t_helmholtz_sweep_noalloc: in-place y sweeps need the workspace of "
                                          "mol_t_helmholtz_sweep (d_in must differ from d_out)");
    size_t tb = 0, jb = 0;
    molt::sweep_scratch_layout(g, precision, batch, &tb, &jb);
    if (tb + jb > kScratchBytes)
      return molt::set_error(MOLT_EUNSUPPORTED,
                             (std::string("mol_t_helmholtz_sweep_noalloc: the y sweep needs ") +
                              std::to_string(tb + jb) + " bytes of scratch, more than its static " +
                              std::to_string(kScratchBytes))
                                 .c_str());
    void* base = nullptr;
    rc = scratch_ptr(&base);
    if (rc != MOLT_OK) return rc;
    tot = base;
    jln = (char*)base + tb;
  }
  return molt::sweep_impl(g, axis, alpha, precision, d_in, d_out, batch, tot, jln, nullptr, (hipStream_t)stream);
}

}  // extern "C"
