// Sub-allocation of the serving arena (host-only; no HIP dependency, so the
// host checks can build it with a plain C++ compiler and sanitizers).
//
// The server reserves one device arena of its memory budget.  Request images
// are placed first-fit from the bottom, the batch workspace last-fit from the
// top, so that the long-lived images and the workspace that is re-planned at
// every membership change grow towards each other.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace gba {

// First-fit from the bottom / last-fit from the top over [0, size).
class RangeAlloc {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc_low(size_t n, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[o + n] = sz - n;
            off = o;
            return true;
        }
        return false;
    }
    bool alloc_high(size_t n, size_t& off) {
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, sz = it->second;
            free_.erase(o);
            if (sz > n) free_[o] = sz - n;
            off = o + sz - n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        if (!n) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto& kv : free_) s += kv.second;
        return s;
    }
    size_t n_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;
};

// Admission check of one request, in the order the server then performs the
// allocations: the image is placed at admission while the current batch
// workspace is still held, and only at the next repack is the workspace
// released and the grown one placed from the top.  Simulated on a copy, so
// the image offset found here is the one the real first-fit returns.
inline bool simulate_admission(const RangeAlloc& ra, bool have_union, size_t union_off,
                               size_t union_bytes, size_t image_bytes, size_t grown_union_bytes,
                               size_t& image_off) {
    RangeAlloc sim = ra;
    size_t io = 0, uo = 0;
    if (!sim.alloc_low(image_bytes, io)) return false;
    if (have_union) sim.release(union_off, union_bytes);
    if (!sim.alloc_high(grown_union_bytes, uo)) return false;
    image_off = io;
    return true;
}

}  // namespace gba
