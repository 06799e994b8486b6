// Host-only building blocks of the batch and server runtime: the arena that
// places admitted requests inside a server's device budget, and the
// assignment of a batch's jobs to streams. Plain C++ (no device calls), so
// they can be built and checked without a GPU.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <cstdint>
#include <map>
#include <numeric>
#include <vector>

namespace hullmi {

// First-fit allocator over offsets [0, size). Free blocks are kept sorted by
// offset and merged with their neighbours on release, so a long run of
// requests of mixed sizes does not fragment the budget permanently.
class Arena {
public:
    static constexpr size_t kNone = SIZE_MAX;

    explicit Arena(size_t size = 0, size_t align = 256) : size_(size), align_(align)
    {
        if (size_ > 0) free_[0] = size_;
    }

    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // Offset of a block of at least `bytes`, or kNone when no free block fits.
    size_t alloc(size_t bytes)
    {
        const size_t need = round(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            live_[off] = need;
            used_ += need;
            if (used_ > peak_) peak_ = used_;
            return off;
        }
        return kNone;
    }

    // Returns the block at `off` (from alloc); false when there is none.
    bool release(size_t off)
    {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t start = off, len = it->second;
        used_ -= len;
        live_.erase(it);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    // Whether a block of `bytes` could be allocated right now.
    bool fits(size_t bytes) const
    {
        const size_t need = round(bytes == 0 ? 1 : bytes);
        for (const auto &f : free_)
            if (f.second >= need) return true;
        return false;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return used_; }
    size_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }
    size_t live_blocks() const { return live_.size(); }

private:
    size_t size_, align_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, never adjacent
    std::map<size_t, size_t> live_;   // offset -> length
};

// Longest-processing-time-first assignment: jobs in decreasing cost go to the
// stream with the least total cost so far (ties to the lower stream index;
// equal costs keep their job order). Returns the stream of every job.
inline std::vector<int> assign_streams(const std::vector<double> &cost, int streams)
{
    std::vector<int> order(cost.size()), out(cost.size(), 0);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(streams > 0 ? streams : 1, 0.0);
    for (int j : order) {
        int best = 0;
        for (int s = 1; s < (int)load.size(); ++s)
            if (load[s] < load[best]) best = s;
        out[j] = best;
        load[best] += cost[j];
    }
    return out;
}

// A byte range [begin, end) that job `job` reads or writes.
struct Span {
    uintptr_t begin, end;
    int job;
    bool write;
};

// Whether ranges of two different jobs overlap where at least one of them is
// written: such jobs race when they run on different streams. Ranges of one
// job are not compared with each other; empty ranges never overlap.
inline bool spans_conflict(std::vector<Span> v)
{
    std::sort(v.begin(), v.end(), [](const Span &a, const Span &b) { return a.begin < b.begin; });
    for (size_t i = 0; i < v.size(); ++i) {
        if (v[i].begin >= v[i].end) continue;
        for (size_t j = i + 1; j < v.size() && v[j].begin < v[i].end; ++j) {
            if (v[j].begin >= v[j].end || v[j].job == v[i].job) continue;
            if (v[i].write || v[j].write) return true;
        }
    }
    return false;
}

}  // namespace hullmi
