// Admission rule of the server (host only, no HIP): which ready requests
// join the batch.
#pragma once
#include <cstddef>
#include <vector>

namespace ep {

// Walking the ready requests in arrival order, admit each one whose device
// footprint still fits the budget (used + footprint <= budget) while a slot
// is free; a request that does not fit stays queued and lets later, smaller
// ones pass.  Returns the positions admitted, in order, and updates `used`.
inline std::vector<size_t> admit_ready(const std::vector<size_t> &footprint, size_t &used,
                                       size_t budget, size_t free_slots) {
    std::vector<size_t> out;
    for (size_t i = 0; i < footprint.size() && out.size() < free_slots; ++i)
        if (footprint[i] <= budget && used <= budget - footprint[i]) {
            used += footprint[i];
            out.push_back(i);
        }
    return out;
}

}  // namespace ep
