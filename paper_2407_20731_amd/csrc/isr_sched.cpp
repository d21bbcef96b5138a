// Batched compression and the request queue behind isr_submit / isr_poll.
#include "isr_sched.h"

#include <chrono>
#include <cstring>

namespace isr {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int run_batch(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st) {
  int first = ISR_OK;
  for (int i = 0; i < count; ++i) {
    int rc = run_compress(c, &fs[i], &outs[i], st ? &st[i] : nullptr);
    if (st) st[i].status = rc;
    if (rc != ISR_OK && first == ISR_OK) first = rc;
  }
  return first;
}

Scheduler::Scheduler(isr_ctx* c) : ctx_(c) { worker_ = std::thread([this] { loop(); }); }

Scheduler::~Scheduler() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (worker_.joinable()) worker_.join();
  for (auto& kv : reqs_)
    if (kv.second.blob) isr_blob_free(kv.second.blob);
}

int Scheduler::submit(const isr_field* f, uint64_t* req) {
  std::lock_guard<std::mutex> g(mu_);
  const uint64_t id = next_id_++;
  Req r;
  r.id = id;
  r.f = *f;
  r.t_submit = now_s();
  std::memset(&r.st, 0, sizeof(r.st));
  reqs_.emplace(id, r);
  queue_.push_back(id);
  *req = id;
  cv_.notify_one();
  return ISR_OK;
}

void Scheduler::loop() {
  for (;;) {
    uint64_t id;
    isr_field f;
    {
      std::unique_lock<std::mutex> g(mu_);
      cv_.wait(g, [&] { return stop_ || !queue_.empty(); });
      if (stop_ && queue_.empty()) return;
      id = queue_.front();
      queue_.pop_front();
      f = reqs_[id].f;
    }
    isr_blob* b = nullptr;
    isr_stats st;
    std::memset(&st, 0, sizeof(st));
    int rc = isr_compress(ctx_, &f, &b, &st);
    {
      std::lock_guard<std::mutex> g(mu_);
      Req& r = reqs_[id];
      r.done = true;
      r.status = rc;
      r.blob = b;
      r.st = st;
      r.st.t_submit = r.t_submit;
    }
    done_cv_.notify_all();
  }
}

int Scheduler::poll(uint64_t req, int wait_ms, isr_blob** out, isr_stats* st) {
  std::unique_lock<std::mutex> g(mu_);
  auto it = reqs_.find(req);
  if (it == reqs_.end()) return ISR_ENOTFOUND;
  if (!it->second.done) {
    if (wait_ms < 0)
      done_cv_.wait(g, [&] { return it->second.done; });
    else if (wait_ms > 0)
      done_cv_.wait_for(g, std::chrono::milliseconds(wait_ms), [&] { return it->second.done; });
    if (!it->second.done) return ISR_PENDING;
  }
  Req r = it->second;
  reqs_.erase(it);
  if (out) *out = r.blob;
  else if (r.blob) isr_blob_free(r.blob);
  if (st) *st = r.st;
  return r.status;
}

}  // namespace isr
