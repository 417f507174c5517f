// Host-only parts of the serving loop that need no device: the first-fit
// arena allocator over the server's device budget and the batch former.
// Plain C++17 so that they can be built and tested without a GPU.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <iterator>
#include <map>
#include <vector>

namespace bbc {

// First-fit allocator of [0, capacity) in 256-byte granules; adjacent free
// ranges are merged on release.  Offsets, not pointers: the caller adds the
// arena's device base address.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  static size_t round(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

  explicit Arena(size_t capacity = 0) { reset(capacity); }

  void reset(size_t capacity) {
    cap_ = capacity & ~(kAlign - 1);
    free_.clear();
    if (cap_) free_[0] = cap_;
    used_ = peak_ = 0;
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  // largest request that can ever succeed (an empty arena)
  bool ever_fits(size_t bytes) const { return round(bytes) <= cap_; }

  // offset of a fresh range of `bytes` (rounded up), or SIZE_MAX if no free
  // range is large enough right now
  size_t alloc(size_t bytes) {
    const size_t b = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      const size_t off = it->first, rest = it->second - b;
      free_.erase(it);
      if (rest) free_[off + b] = rest;
      used_ += b;
      if (used_ > peak_) peak_ = used_;
      return off;
    }
    return SIZE_MAX;
  }

  void release(size_t off, size_t bytes) {
    const size_t b = round(bytes ? bytes : 1);
    used_ -= b;
    auto next = free_.lower_bound(off);
    size_t start = off, len = b;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && next->first == off + b) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }

  size_t n_free_ranges() const { return free_.size(); }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& r : free_) m = r.second > m ? r.second : m;
    return m;
  }

 private:
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

// A request waiting for admission, as the batch former sees it.
struct PendingView {
  int32_t scene;
  int64_t n;
};

// Choose the requests of the next batch from the pending queue (in arrival
// order): the oldest request fixes the scene; later requests of the same
// scene join while the batch stays within max_points points and max_reqs
// requests and its device need (need(points, requests)) still fits `fits`.
// Requests of other scenes keep their place.  Returns indices into `queue`;
// empty when even the oldest request does not fit right now.
inline std::vector<size_t> form_batch(const std::vector<PendingView>& queue, int64_t max_points, int32_t max_reqs,
                                      const std::function<size_t(int32_t scene, int64_t points, int32_t reqs)>& need,
                                      const std::function<bool(size_t bytes)>& fits) {
  std::vector<size_t> pick;
  if (queue.empty()) return pick;
  const int32_t scene = queue[0].scene;
  int64_t pts = 0;
  for (size_t k = 0; k < queue.size(); ++k) {
    if (queue[k].scene != scene) continue;
    if (int32_t(pick.size()) >= max_reqs) break;
    const int64_t p2 = pts + queue[k].n;
    if (p2 > max_points) {
      if (pick.empty()) return pick;  // the oldest request alone exceeds the batch size
      continue;
    }
    if (!fits(need(scene, p2, int32_t(pick.size()) + 1))) {
      if (pick.empty()) return pick;
      continue;
    }
    pick.push_back(k);
    pts = p2;
  }
  return pick;
}

// Percentile of a sample (linear interpolation between order statistics).
inline double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double r = q / 100.0 * double(v.size() - 1);
  const size_t lo = size_t(r);
  const size_t hi = lo + 1 < v.size() ? lo + 1 : lo;
  return v[lo] + (r - double(lo)) * (v[hi] - v[lo]);
}

}  // namespace bbc
