// Host-side device queries shared by the launchers, cached per device.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>

namespace pecc {

constexpr int kMaxDevices = 64;

// Compute units of the current device (256 if the query fails).  Cached per
// device; concurrent first calls store the same value.
inline int current_device_cus()
{
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    int c = dev < kMaxDevices ? cache[dev].load(std::memory_order_relaxed) : 0;
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        if (dev < kMaxDevices) cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// Resident workgroups per CU of `kernel` at `threads` per workgroup on the
// current device (1 if the query fails), cached per device in `cache`.
template <typename K>
inline int resident_per_cu(K kernel, int threads, std::atomic<int> (&cache)[kMaxDevices])
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 1;
    int c = dev < kMaxDevices ? cache[dev].load(std::memory_order_relaxed) : 0;
    if (c <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, kernel, threads, 0) != hipSuccess ||
            c <= 0)
            c = 1;
        if (dev < kMaxDevices) cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

}  // namespace pecc
