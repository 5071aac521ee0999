// The per-request copy for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that must not call the allocator):
// devirt_copy_static.  It runs the kernels of devirt_copy_from_guest /
// devirt_copy_to_guest, with the scratch those kernels need -- one request's
// epoch counters, the clock origin and the long and short segment queues --
// in a static device array instead of the stream's workspace.
//
// Every device the library runs on holds one copy of the array until the
// process ends.  Calls on one device share it and it keeps the last call's
// contents: the translate kernel clears the queue counters itself (a kernel,
// so the call can be captured), and calls that overlap on one device race.
#include <cerrno>
#include <mutex>

#include "runtime.h"

using namespace dv;

namespace {

// Requests touching at most this many 4 KiB pages (64 MiB): one queued
// segment per page in the long or the short queue.
constexpr uint64_t kStaticPages = 16384;
constexpr size_t kCtrBytes = (sizeof(DEpochCtr) + 255) & ~size_t(255);
constexpr size_t kT0Bytes = 256;
constexpr size_t kQueueBytes = kStaticPages * sizeof(DSeg);
constexpr size_t kScratchBytes = kCtrBytes + kT0Bytes + 2 * kQueueBytes;  // about 1 MiB

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // the array's device address, per device (null: not looked up yet)

}  // namespace

// Called by devirt_open with `device` current.  The array's host-side name is
// not a device address: the address is looked up once per device and only
// that address is used afterwards.
int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return dv_fail(-EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return 0;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return dv_fail(-EIO, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_ptr[device] = p;
    return 0;
}

extern "C" int devirt_copy_static(devirt_ctx *c, uint32_t asid, uint64_t gva, void *host_dev, uint64_t len,
                                  uint32_t dir, devirt_result *res_dev, void *hip_stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (dir != DEVIRT_FROM_GUEST && dir != DEVIRT_TO_GUEST) return dv_fail(-EINVAL, "dir must be 0 or 1");
    void *base;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = (c->device >= 0 && c->device < kMaxDevices) ? g_ptr[c->device] : nullptr;
    }
    if (!base) return dv_fail(-EIO, "no static scratch on device %d", c->device);
    uint8_t *p = (uint8_t *)base;
    StaticScratch st;
    st.ctr = (DEpochCtr *)p;
    st.t0 = (uint64_t *)(p + kCtrBytes);
    st.segs = (DSeg *)(p + kCtrBytes + kT0Bytes);
    st.shorts = (DSeg *)(p + kCtrBytes + kT0Bytes + kQueueBytes);
    st.cap = kStaticPages;
    return plain_copy(c, asid, gva, (uint64_t)(uintptr_t)host_dev, len, dir, res_dev, hip_stream, &st);
}
