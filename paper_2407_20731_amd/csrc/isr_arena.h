// Host-only pieces of the runtime that carry no device code: the budgeted
// sub-allocator behind every device allocation of a context, and the FIFO
// admission rule of the scheduler.  Both are plain C++ (no HIP types), so
// they build and are tested on the CPU with fake device memory.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

namespace isr {

// Sub-allocator over large chunks taken from a device allocator, capped by a
// budget: first fit for short-lived scratch, top of the highest free range
// for long-lived blobs, coalescing of freed ranges, in-place shrink, and
// chunks with nothing live handed back when the budget is held in ranges too
// small for a request.  Thread-safe.
class Arena {
 public:
  typedef void* (*ChunkAlloc)(size_t bytes, void* user);  // nullptr on failure
  typedef void (*ChunkFree)(void* p, void* user);
  Arena(uint64_t budget, ChunkAlloc ca, ChunkFree cf, void* user, size_t chunk_bytes = (size_t)256 << 20);
  ~Arena();
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  // 256-byte granules; nullptr when the budget or the device is exhausted.
  void* alloc(size_t bytes, bool high = false);
  void free(void* p);  // unknown pointers are ignored
  void shrink(void* p, size_t bytes);
  void release();      // every chunk back to the device allocator
  uint64_t budget() const { return budget_; }
  uint64_t used() const;
  uint64_t held() const;
  uint64_t high_water() const;
  size_t live_count() const;

 private:
  struct Chunk {
    char* base;
    size_t size;
    std::map<size_t, size_t> free;  // offset -> length
  };
  void give_back(int ci, size_t off, size_t sz);
  mutable std::mutex mu_;
  ChunkAlloc ca_;
  ChunkFree cf_;
  void* user_;
  size_t chunk_bytes_;
  uint64_t budget_, held_ = 0, used_ = 0, high_ = 0;
  std::vector<Chunk> chunks_;
  std::map<char*, std::pair<int, size_t>> live_;
};

// Start queued requests in FIFO order while a slot is free.  Slots need
// members `busy` and `id`.  start(slot, id) begins request id on that slot
// and returns 0 (started), kENoMem or another error code.  A request that
// does not fit while others run stays at the head of the queue (it waits for
// them to free memory; later requests wait behind it, so none starves); with
// nothing running it cannot fit at all and ends with kENoMem, as do requests
// failing with any other code (end(id, code)).  *running_high keeps the
// largest number of requests running at once.  Returns true when a request
// started or ended.
template <class SlotVec, class Start, class End>
bool admit_fifo(std::deque<uint64_t>& queue, SlotVec& slots, int kENoMem, Start start, End end,
                uint64_t* running_high) {
  bool any = false;
  while (!queue.empty()) {
    auto* free_slot = static_cast<decltype(&slots[0])>(nullptr);
    for (auto& s : slots)
      if (!s.busy) {
        free_slot = &s;
        break;
      }
    if (!free_slot) break;
    const uint64_t id = queue.front();
    const int rc = start(*free_slot, id);
    if (rc == kENoMem) {
      bool running = false;
      for (auto& s : slots) running = running || s.busy;
      if (running) break;
    }
    queue.pop_front();
    any = true;
    if (rc != 0) {
      end(id, rc);
      continue;
    }
    free_slot->busy = true;
    free_slot->id = id;
    uint64_t n = 0;
    for (auto& s : slots) n += s.busy ? 1 : 0;
    if (running_high && n > *running_high) *running_high = n;
  }
  return any;
}

}  // namespace isr
