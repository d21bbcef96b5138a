// Budgeted sub-allocator (declared in isr_arena.h).  Host code only.
#include "isr_arena.h"

#include <algorithm>

namespace isr {

Arena::Arena(uint64_t budget, ChunkAlloc ca, ChunkFree cf, void* user, size_t chunk_bytes)
    : ca_(ca), cf_(cf), user_(user), chunk_bytes_(chunk_bytes ? chunk_bytes : 256), budget_(budget) {}

Arena::~Arena() { release(); }

void Arena::release() {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& c : chunks_)
    if (c.base) cf_(c.base, user_);
  chunks_.clear();
  live_.clear();
  held_ = 0;
  used_ = 0;
}

uint64_t Arena::used() const {
  std::lock_guard<std::mutex> g(mu_);
  return used_;
}

uint64_t Arena::held() const {
  std::lock_guard<std::mutex> g(mu_);
  return held_;
}

uint64_t Arena::high_water() const {
  std::lock_guard<std::mutex> g(mu_);
  return high_;
}

size_t Arena::live_count() const {
  std::lock_guard<std::mutex> g(mu_);
  return live_.size();
}

void* Arena::alloc(size_t bytes, bool high) {
  std::lock_guard<std::mutex> g(mu_);
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  // low: first fitting range in address order; high: the last one
  int best_c = -1;
  size_t best_off = 0, best_sz = 0;
  for (size_t ci = 0; ci < chunks_.size(); ++ci)
    for (auto& fr : chunks_[ci].free)
      if (fr.second >= bytes && (best_c < 0 || high)) {
        best_c = (int)ci;
        best_off = fr.first;
        best_sz = fr.second;
      }
  if (best_c < 0) {
    // a new chunk: chunk_bytes_, or what is left of the budget, or at least `bytes`
    auto wanted = [&] {
      return std::max(bytes, std::min(chunk_bytes_, (size_t)(budget_ > held_ ? budget_ - held_ : 0)));
    };
    size_t want = wanted();
    if (held_ + want > budget_) {
      // the budget is held in ranges too small for this request: give the
      // chunks with nothing live in them back to the device and try again
      for (auto& c : chunks_)
        if (c.base && c.free.size() == 1 && c.free.begin()->first == 0 && c.free.begin()->second == c.size) {
          cf_(c.base, user_);
          held_ -= c.size;
          c.base = nullptr;
          c.size = 0;
          c.free.clear();
        }
      want = wanted();
      if (held_ + want > budget_) return nullptr;
    }
    void* p = ca_(want, user_);
    if (!p) return nullptr;
    Chunk c;
    c.base = (char*)p;
    c.size = want;
    c.free[0] = want;
    best_c = -1;
    for (size_t ci = 0; ci < chunks_.size() && best_c < 0; ++ci)
      if (!chunks_[ci].base) best_c = (int)ci;  // reuse a released slot (live_ keeps indices)
    if (best_c < 0) {
      chunks_.push_back(c);
      best_c = (int)chunks_.size() - 1;
    } else {
      chunks_[best_c] = c;
    }
    held_ += want;
    best_off = 0;
    best_sz = want;
  }
  Chunk& c = chunks_[best_c];
  c.free.erase(best_off);
  size_t at = best_off;
  if (high) {
    at = best_off + best_sz - bytes;
    if (best_sz > bytes) c.free[best_off] = best_sz - bytes;
  } else if (best_sz > bytes) {
    c.free[best_off + bytes] = best_sz - bytes;
  }
  char* p = c.base + at;
  live_[p] = {best_c, bytes};
  used_ += bytes;
  high_ = std::max(high_, used_);
  return p;
}

void Arena::give_back(int ci, size_t off, size_t sz) {
  Chunk& c = chunks_[ci];
  auto it = c.free.emplace(off, sz).first;
  // merge with the next range
  auto nx = std::next(it);
  if (nx != c.free.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    c.free.erase(nx);
  }
  // merge with the previous range
  if (it != c.free.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      c.free.erase(it);
    }
  }
}

void Arena::free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  auto it = live_.find((char*)p);
  if (it == live_.end()) return;
  int ci = it->second.first;
  size_t sz = it->second.second;
  size_t off = (char*)p - chunks_[ci].base;
  live_.erase(it);
  used_ -= sz;
  give_back(ci, off, sz);
}

void Arena::shrink(void* p, size_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = live_.find((char*)p);
  if (it == live_.end()) return;
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  size_t old = it->second.second;
  if (bytes >= old) return;
  int ci = it->second.first;
  size_t off = (char*)p - chunks_[ci].base;
  it->second.second = bytes;
  used_ -= old - bytes;
  give_back(ci, off + bytes, old - bytes);
}

}  // namespace isr
