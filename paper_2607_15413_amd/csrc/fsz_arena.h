// First-fit allocator over a fixed byte range, used by the served form to
// admit requests against a device-memory budget.  Host-only bookkeeping: it
// hands out offsets, the caller adds them to its device base pointer.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace fsz {

class Arena {
public:
    static constexpr uint64_t kAlign = 256;

    explicit Arena(uint64_t size = 0) { reset(size); }

    void reset(uint64_t size)
    {
        size_ = size / kAlign * kAlign;
        free_.clear();
        live_.clear();
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }

    static uint64_t round_up(uint64_t n) { return (n ? (n + kAlign - 1) / kAlign : 1) * kAlign; }

    // whether a request of n bytes could ever be admitted
    bool fits_ever(uint64_t n) const { return round_up(n) <= size_; }

    // Lowest-offset free range that holds n bytes; false when none does.
    bool alloc(uint64_t n, uint64_t *off)
    {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const uint64_t rest = it->second - n;
            const uint64_t start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            live_[*off] = n;
            used_ += n;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }

    // Frees the allocation starting at off (merging with free neighbours);
    // false if no allocation starts there.
    bool release(uint64_t off)
    {
        auto l = live_.find(off);
        if (l == live_.end()) return false;
        uint64_t n = l->second;
        live_.erase(l);
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return true;
            }
        }
        free_[off] = n;
        return true;
    }

    bool is_live(uint64_t off) const { return live_.count(off) != 0; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t size() const { return size_; }
    uint64_t free_ranges() const { return free_.size(); }

    // Invariants: free and live ranges tile [0, size) without overlap, free
    // ranges are never adjacent, and used() is the sum of live ranges.
    bool check() const
    {
        std::map<uint64_t, std::pair<uint64_t, bool>> all;
        for (auto &f : free_) all[f.first] = {f.second, true};
        for (auto &l : live_) {
            if (all.count(l.first)) return false;
            all[l.first] = {l.second, false};
        }
        uint64_t pos = 0, live_sum = 0;
        bool prev_free = false;
        for (auto &a : all) {
            if (a.first != pos || a.second.first == 0 || a.second.first % kAlign) return false;
            if (a.second.second && prev_free) return false;
            prev_free = a.second.second;
            if (!a.second.second) live_sum += a.second.first;
            pos += a.second.first;
        }
        return pos == size_ && live_sum == used_;
    }

private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    std::map<uint64_t, uint64_t> live_;  // offset -> bytes
};

}  // namespace fsz
