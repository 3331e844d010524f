// Host helper: how many workgroups of a kernel are resident on the whole
// chip at once (the grid of a persistent launch).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>

namespace sgs {

// workgroups of `kernel` resident at once over all CUs (cached per device,
// kernel and dynamic LDS size); 0 if the runtime cannot say
template <typename K>
int64_t resident_blocks(K kernel, int threads, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_tuple(dev, reinterpret_cast<const void*>(kernel), lds);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int64_t r = (int64_t)(per_cu < 1 ? 1 : per_cu) * (cus < 1 ? 1 : cus);
    cache[key] = r;
    return r;
}

}  // namespace sgs
