// Allocation-free operator application (ovs_apply_noalloc): ovs_apply's two
// staging fields live in a fixed per-device scratch array instead of the
// handle's workspace, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ovs_common.h"
#include "ovs_host.h"

namespace ovs {
constexpr size_t kNoAllocScratchBytes = OVS_APPLY_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace ovs

// One copy per GPU that loads the library, kept until the process ends.  In
// host code this name is a stand-in, not a device address: host code uses
// only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[ovs::kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[ovs::kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch, resolved once per device with that
// device current (the caller's current device is restored).
static ovs_status scratch_address(int device, void** out) {
  if (device < 0 || device >= ovs::kMaxDevices) return OVS_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    OVS_HIP(hipGetDevice(&cur));
    if (cur != device) OVS_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      ovs::record_error("hipGetSymbolAddress(scratch)", __LINE__, e != hipSuccess ? e : hipErrorInvalidSymbol);
      return OVS_ERR_HIP;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return OVS_OK;
}

extern "C" ovs_status ovs_apply_noalloc(ovs_lattice l, ovs_op op, const void* x, void* y,
                                        int32_t nrhs) {
  using namespace ovs;
  if (!l || !x || !y || x == y || nrhs < 1 || nrhs > kMaxNrhs || op < 0 || op > 3)
    return OVS_ERR_ARG;
  if (!ready(l)) return OVS_ERR_STATE;
  const size_t fb = (size_t)nrhs * 12 * l->g.Vs * elem_bytes(l);
  const size_t fb_al = (fb + 255) & ~size_t(255);
  if (2 * fb_al > kNoAllocScratchBytes) return OVS_ERR_ARG;
  void* base = nullptr;
  ovs_status st = scratch_address(l->device, &base);
  if (st != OVS_OK) return st;
  StreamScope sc(l);
  void* fin = base;
  void* fout = (char*)base + fb_al;
  Hop h;
  bool g5in, g5out;
  op_setup(l, op, h, g5in, g5out);
  pack_field(l, x, fin, nrhs);
  OVS_HIP(launch_wilson(l->prec == OVS_F32_STORE, l->links, fin, fout, nrhs, l->g, h, g5in, g5out,
                        get_tuning(l, nrhs), l->stream));
  unpack_field(l, fout, y, nrhs);
  OVS_HIP(hipGetLastError());
  return OVS_OK;
}
