// CPU tests of the runtime's host-only pieces (paper_2407_20731_amd/csrc/
// isr_arena.h): the budgeted sub-allocator over fake device chunks (malloc,
// so AddressSanitizer sees every byte), and the scheduler's FIFO admission
// rule against a fake executor with its own memory budget.  Built with
// -fsanitize=address,undefined by tests/test_arena_admit_cpu.py; exits 0 and
// prints "ALL OK" when every check holds.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "isr_arena.h"

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "%s:%d: CHECK(%s) failed\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

// ---- fake device allocator ------------------------------------------------
struct FakeDev {
  std::map<void*, size_t> chunks;  // outstanding
  size_t allocs = 0, frees = 0;
  long fail_after = -1;            // fail the n-th allocation (0-based) and later
  std::mutex mu;
};

static void* fake_alloc(size_t bytes, void* u) {
  FakeDev* d = (FakeDev*)u;
  std::lock_guard<std::mutex> g(d->mu);
  if (d->fail_after >= 0 && (long)d->allocs >= d->fail_after) return nullptr;
  void* p = std::malloc(bytes);
  if (!p) return nullptr;
  std::memset(p, 0xCD, bytes);
  d->chunks[p] = bytes;
  ++d->allocs;
  return p;
}

static void fake_free(void* p, void* u) {
  FakeDev* d = (FakeDev*)u;
  std::lock_guard<std::mutex> g(d->mu);
  auto it = d->chunks.find(p);
  if (it == d->chunks.end()) {
    std::fprintf(stderr, "free of an unknown chunk\n");
    ++g_fail;
    return;
  }
  d->chunks.erase(it);
  ++d->frees;
  std::free(p);
}

// every live range lies inside one outstanding chunk, and no two overlap
static void check_ranges(FakeDev& d, const std::map<char*, size_t>& live) {
  char* prev_end = nullptr;
  for (auto& kv : live) {
    CHECK(kv.first >= prev_end);
    prev_end = kv.first + kv.second;
    bool inside = false;
    for (auto& c : d.chunks)
      if (kv.first >= (char*)c.first && kv.first + kv.second <= (char*)c.first + c.second) inside = true;
    CHECK(inside);
  }
}

static void test_arena_basics() {
  FakeDev d;
  {
    isr::Arena a(1 << 20, fake_alloc, fake_free, &d, 64 << 10);
    char* p = (char*)a.alloc(1);
    CHECK(p && a.used() == 256 && a.held() == (64 << 10));
    char* q = (char*)a.alloc(300);
    CHECK(q == p + 256 && a.used() == 256 + 512);  // first fit, 256-byte granules
    char* r = (char*)a.alloc(1000);
    CHECK(r == q + 512);
    a.free(q);
    a.free(p);  // p and q coalesce into [0, 768)
    char* s = (char*)a.alloc(768);
    CHECK(s == p);
    // a long-lived allocation takes the top of the highest free range
    char* h = (char*)a.alloc(4096, true);
    CHECK(h == p + (64 << 10) - 4096);
    // shrink in place: the tail is free again
    a.shrink(r, 256);
    char* t = (char*)a.alloc(512);
    CHECK(t == r + 256);
    a.free((void*)0x1234);  // unknown pointers are ignored
    a.free(nullptr);
    CHECK(a.live_count() == 4);
    a.free(s);
    a.free(h);
    a.free(r);
    a.free(t);
    CHECK(a.used() == 0 && a.high_water() >= 256 + 512 + 1024);
  }
  CHECK(d.chunks.empty() && d.allocs == d.frees);
}

static void test_arena_budget_and_release() {
  FakeDev d;
  isr::Arena a(256 << 10, fake_alloc, fake_free, &d, 64 << 10);
  std::vector<void*> v;
  for (int i = 0; i < 4; ++i) v.push_back(a.alloc(64 << 10));
  CHECK(v[3] != nullptr && a.held() == (256 << 10));
  CHECK(a.alloc(256) == nullptr);  // the budget is held
  a.free(v[1]);
  a.free(v[2]);
  // 128 KiB free in two chunks: a request larger than a chunk needs the
  // empty chunks handed back and one new chunk of its size
  void* big = a.alloc(100 << 10);
  CHECK(big != nullptr && a.held() <= (256 << 10));
  CHECK(d.frees >= 2);
  CHECK(a.alloc(200 << 10) == nullptr);  // more than the budget can hold now
  a.free(big);
  a.free(v[0]);
  a.free(v[3]);
  CHECK(a.used() == 0);
  void* whole = a.alloc(256 << 10);  // the whole budget in one range
  CHECK(whole != nullptr);
  a.free(whole);
  a.release();
  CHECK(d.chunks.empty() && a.held() == 0 && a.live_count() == 0);
  // device allocator failures: nullptr and nothing held
  FakeDev f;
  f.fail_after = 1;
  isr::Arena b(1 << 20, fake_alloc, fake_free, &f, 64 << 10);
  void* x = b.alloc(1000);
  CHECK(x != nullptr);
  CHECK(b.alloc(100 << 10) == nullptr && b.held() == (64 << 10));
  b.free(x);
}

static void test_arena_random() {
  std::mt19937_64 rng(7);
  for (int round = 0; round < 20; ++round) {
    FakeDev d;
    const uint64_t budget = (1 + rng() % 16) << 16;
    isr::Arena a(budget, fake_alloc, fake_free, &d, (1 + rng() % 4) << 14);
    std::map<char*, size_t> live;
    for (int op = 0; op < 4000; ++op) {
      const int kind = (int)(rng() % 10);
      if (kind < 5 || live.empty()) {
        const size_t want = 1 + rng() % (rng() % 4 == 0 ? 40000 : 3000);
        const bool high = rng() % 3 == 0;
        char* p = (char*)a.alloc(want, high);
        if (p) {
          const size_t g = (want + 255) & ~size_t(255);
          std::memset(p, op & 0xFF, g);  // the whole range is ours (ASan checks the chunk bounds)
          live[p] = g;
        } else {
          // refusal only when the budget cannot hold it
          uint64_t used = 0;
          for (auto& kv : live) used += kv.second;
          CHECK(used + ((want + 255) & ~size_t(255)) > budget || a.held() + ((want + 255) & ~size_t(255)) > budget);
        }
      } else if (kind < 9) {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        a.free(it->first);
        live.erase(it);
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        const size_t nb = 1 + rng() % it->second;
        a.shrink(it->first, nb);
        it->second = std::min(it->second, (nb + 255) & ~size_t(255));
      }
      uint64_t used = 0;
      for (auto& kv : live) used += kv.second;
      CHECK(a.used() == used);
      CHECK(a.held() <= budget);
      if (op % 97 == 0) check_ranges(d, live);
    }
    check_ranges(d, live);
    for (auto& kv : live) a.free(kv.first);
    CHECK(a.used() == 0);
    a.release();
    CHECK(d.chunks.empty());
  }
}

static void test_arena_threads() {
  FakeDev d;
  isr::Arena a(64ull << 20, fake_alloc, fake_free, &d, 1 << 20);
  std::vector<std::thread> th;
  for (int t = 0; t < 8; ++t)
    th.emplace_back([&a, t] {
      std::mt19937_64 rng(100 + t);
      std::vector<std::pair<char*, size_t>> mine;
      for (int op = 0; op < 3000; ++op) {
        if (mine.empty() || rng() % 2) {
          const size_t n = 1 + rng() % 20000;
          char* p = (char*)a.alloc(n, rng() % 2);
          if (p) {
            std::memset(p, t, n);
            mine.push_back({p, n});
          }
        } else {
          const size_t k = rng() % mine.size();
          a.free(mine[k].first);
          mine[k] = mine.back();
          mine.pop_back();
        }
      }
      for (auto& m : mine) a.free(m.first);
    });
  for (auto& x : th) x.join();
  CHECK(a.used() == 0 && a.live_count() == 0);
}

// ---- admission against a fake executor -------------------------------------
struct FakeSlot {
  bool busy = false;
  uint64_t id = 0;
};

static void run_admission(int nslots, uint64_t budget, const std::vector<uint64_t>& fp,
                          const std::vector<int>& bad, uint64_t seed) {
  const int kENoMem = -2, kEInval = -1;
  std::deque<uint64_t> queue;
  for (uint64_t i = 0; i < fp.size(); ++i) queue.push_back(i);
  std::vector<FakeSlot> slots(nslots);
  uint64_t used = 0, high = 0;
  std::vector<int> status(fp.size(), 1);  // 1 = pending
  std::vector<uint64_t> order;            // ids in the order they left the queue
  std::mt19937_64 rng(seed);
  auto start = [&](FakeSlot&, uint64_t id) {
    if (std::find(bad.begin(), bad.end(), (int)id) != bad.end()) return kEInval;
    if (used + fp[id] > budget) return kENoMem;
    used += fp[id];
    order.push_back(id);  // started
    return 0;
  };
  auto end = [&](uint64_t id, int rc) {
    status[id] = rc;
    order.push_back(id);
  };
  size_t guard = 0;
  for (;;) {
    isr::admit_fifo(queue, slots, kENoMem, start, end, &high);
    CHECK(used <= budget);
    int running = 0;
    for (auto& s : slots) running += s.busy;
    CHECK((uint64_t)running <= high && high <= (uint64_t)nslots);
    if (queue.empty() && running == 0) break;
    if (running == 0) {
      // nothing runs and the head did not start: it must have been ended
      CHECK(queue.empty());
      break;
    }
    // finish one running request
    std::vector<int> busy;
    for (int k = 0; k < nslots; ++k)
      if (slots[k].busy) busy.push_back(k);
    FakeSlot& s = slots[busy[rng() % busy.size()]];
    used -= fp[s.id];
    status[s.id] = 0;
    s.busy = false;
    CHECK(++guard < 100000);
    if (guard >= 100000) break;
  }
  // every request left the queue exactly once, in FIFO order
  CHECK(order.size() == fp.size());
  for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == i);
  for (uint64_t i = 0; i < fp.size(); ++i) {
    const bool is_bad = std::find(bad.begin(), bad.end(), (int)i) != bad.end();
    if (is_bad)
      CHECK(status[i] == kEInval);
    else if (fp[i] > budget)
      CHECK(status[i] == kENoMem);  // cannot fit even alone: ended, not starved
    else
      CHECK(status[i] == 0);
  }
  CHECK(used == 0);
}

static void test_admission() {
  // two slots, small budget: head-of-line waiting and FIFO
  run_admission(2, 100, {60, 60, 30, 30, 90, 10}, {}, 1);
  // more slots than memory allows, requests larger than the whole budget, errors
  run_admission(8, 1000, {400, 2000, 400, 300, 5000, 100, 999, 1}, {3}, 2);
  // random mixes
  std::mt19937_64 rng(3);
  for (int t = 0; t < 200; ++t) {
    const int n = 1 + (int)(rng() % 40);
    std::vector<uint64_t> fp;
    for (int i = 0; i < n; ++i) fp.push_back(1 + rng() % 300);
    std::vector<int> bad;
    if (rng() % 3 == 0) bad.push_back((int)(rng() % n));
    run_admission(1 + (int)(rng() % 8), 50 + rng() % 400, fp, bad, rng());
  }
  // no slot: nothing starts and the queue is untouched
  std::deque<uint64_t> q = {0, 1};
  std::vector<FakeSlot> none;
  uint64_t high = 0;
  const bool any = isr::admit_fifo(q, none, -2, [](FakeSlot&, uint64_t) { return 0; }, [](uint64_t, int) {}, &high);
  CHECK(!any && q.size() == 2 && high == 0);
}

int main() {
  test_arena_basics();
  test_arena_budget_and_release();
  test_arena_random();
  test_arena_threads();
  test_admission();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
