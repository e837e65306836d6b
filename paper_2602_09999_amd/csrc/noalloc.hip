// Allocation-free form of the pair sort (fgs_sort_pairs_noalloc): the sort's
// scratch (the second key and value buffers of the ping-pong passes and the
// digit histograms) is a static device array of a fixed size instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// Host code never passes the array's name to a kernel or a copy: the name is
// a host-side stand-in.  The array's device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and that address
// is what the sort receives.
#include <mutex>

#include "fgs_internal.h"

namespace {

// Largest sort workspace of FGS_SORT_NOALLOC_MAX_PAIRS pairs (32-bit keys:
// 4 MiB of keys, 4 MiB of values and the histograms of 256 blocks) rounded
// up; fgs_sort_pairs_noalloc checks the exact need against it on every call.
constexpr size_t kScratchBytes = FGS_SORT_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// Device address of the array on `dev`, which must be the current device.
fgs_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fgs::fail(FGS_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fgs::fail(FGS_ERR_HIP, "hipGetSymbolAddress of the sort scratch on device %d: %s", dev,
                       hipGetErrorString(e));
    if ((uintptr_t)p % 256) return fgs::fail(FGS_ERR_HIP, "sort scratch on device %d is not 256-byte aligned", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FGS_OK;
}

}  // namespace

extern "C" fgs_status fgs_sort_pairs_noalloc(void* keys, uint32_t* vals, int64_t n, int32_t key_bytes,
                                             int32_t key_bits, void* stream) {
  if (n < 0 || n > FGS_SORT_NOALLOC_MAX_PAIRS)
    return fgs::fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld not in 0..%d (the static scratch holds %d pairs)",
                     (long long)n, FGS_SORT_NOALLOC_MAX_PAIRS, FGS_SORT_NOALLOC_MAX_PAIRS);
  if (key_bytes != 2 && key_bytes != 4) return fgs::fail(FGS_ERR_INVALID_ARGUMENT, "key_bytes must be 2 or 4");
  if (key_bits < 0 || key_bits > 8 * key_bytes)
    return fgs::fail(FGS_ERR_INVALID_ARGUMENT, "key_bits %d not in 0..%d", key_bits, 8 * key_bytes);
  if (n == 0 || key_bits == 0) return FGS_OK;
  if (!keys || !vals) return fgs::fail(FGS_ERR_INVALID_ARGUMENT, "NULL pointer");
  size_t need = 0;
  fgs_status s = fgs_sort_workspace_size(n, key_bytes, &need);
  if (s != FGS_OK) return s;
  if (need > kScratchBytes)
    return fgs::fail(FGS_ERR_HIP, "internal: %zu scratch bytes needed, %zu reserved", need, kScratchBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fgs::fail(FGS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (hs != nullptr) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(hs, &sdev);
    if (e != hipSuccess) return fgs::fail(FGS_ERR_HIP, "hipStreamGetDevice: %s", hipGetErrorString(e));
    if (sdev != dev)
      return fgs::fail(FGS_ERR_INVALID_ARGUMENT, "stream belongs to device %d, the current device is %d", (int)sdev,
                       dev);
  }
  void* ws = nullptr;
  s = scratch_on(dev, &ws);
  if (s != FGS_OK) return s;
  return fgs_sort_pairs(keys, vals, n, key_bytes, key_bits, ws, kScratchBytes, stream);
}
