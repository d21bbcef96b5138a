// Batched compression and the continuous-batching request scheduler behind
// isr_submit / isr_poll.
#include "isr_sched.h"

#include <chrono>
#include <cstring>

namespace isr {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int run_batch_sequential(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st) {
  int first = ISR_OK;
  for (int i = 0; i < count; ++i) {
    int rc = run_compress(c, &fs[i], &outs[i], st ? &st[i] : nullptr);
    if (st) st[i].status = rc;
    if (rc != ISR_OK && first == ISR_OK) first = rc;
  }
  return first;
}

Scheduler::Scheduler(isr_ctx* c) : ctx_(c) {
  const int n = ctx_max_inflight(c);
  slots_.resize(n);
  (void)hipSetDevice(ctx_device(c));
  for (auto& s : slots_) (void)hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking);  // default priority
  worker_ = std::thread([this] { loop(); });
}

Scheduler::~Scheduler() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (worker_.joinable()) worker_.join();
  (void)hipSetDevice(ctx_device(ctx_));
  for (auto& s : slots_) {
    if (s.busy) {
      (void)hipStreamSynchronize(s.s);
      task_release(&s.t);
    }
    (void)hipStreamDestroy(s.s);
  }
  for (auto& kv : reqs_) {
    if (kv.second.blob) isr_blob_free(kv.second.blob);
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  }
}

int Scheduler::submit(const isr_field* f, uint64_t* req) {
  const uint64_t fp = request_footprint(f);
  if (fp > ctx_budget(ctx_)) return ISR_ENOMEM;
  Req r;
  r.f = *f;
  r.t_submit = now_s();
  std::memset(&r.st, 0, sizeof(r.st));
  // the field is ready once the producer's stream reaches this point
  if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r.ready, (hipStream_t)f->stream) != hipSuccess) {
    if (r.ready) (void)hipEventDestroy(r.ready);
    return ISR_EDEVICE;
  }
  {
    std::lock_guard<std::mutex> g(mu_);
    r.id = next_id_++;
    *req = r.id;
    queue_.push_back(r.id);
    reqs_.emplace(r.id, r);
  }
  cv_.notify_one();
  return ISR_OK;
}

// Start queued requests (FIFO) while a stream slot and HBM budget are free.
bool Scheduler::admit_locked() {
  bool any = false;
  while (!queue_.empty()) {
    Slot* free_slot = nullptr;
    for (auto& s : slots_)
      if (!s.busy) {
        free_slot = &s;
        break;
      }
    if (!free_slot) break;
    const uint64_t id = queue_.front();
    Req& r = reqs_[id];
    (void)hipStreamWaitEvent(free_slot->s, r.ready, 0);
    free_slot->t = Task();
    const int rc = task_begin(ctx_, &r.f, free_slot->s, false, &free_slot->t);
    if (rc == ISR_ENOMEM) {
      bool running = false;
      for (auto& s : slots_) running = running || s.busy;
      if (running) break;  // wait until running requests free memory
    }
    queue_.pop_front();
    if (rc != ISR_OK) {
      r.done = true;
      r.status = rc;
      any = true;
      continue;
    }
    free_slot->busy = true;
    free_slot->id = id;
    any = true;
    uint64_t running = 0;
    for (auto& s : slots_) running += s.busy;
    if (running > high_) high_ = running;
  }
  return any;
}

void Scheduler::loop() {
  (void)hipSetDevice(ctx_device(ctx_));
  std::unique_lock<std::mutex> g(mu_);
  for (;;) {
    bool progressed = admit_locked();
    bool busy = false;
    for (auto& s : slots_) {
      if (!s.busy) continue;
      busy = true;
      const hipError_t q = hipEventQuery(s.t.done);
      if (q == hipErrorNotReady) continue;
      Req& r = reqs_[s.id];
      isr_blob* b = nullptr;
      int rc;
      if (q != hipSuccess) {
        rc = ISR_EDEVICE;
        task_release(&s.t);
      } else {
        rc = task_step(&s.t, &b);
        if (rc == ISR_PENDING) continue;  // repair pass enqueued
      }
      r.done = true;
      r.status = rc;
      r.blob = b;
      r.st = s.t.st;
      r.st.t_submit = r.t_submit;
      r.st.status = rc;
      s.busy = false;
      progressed = true;
    }
    if (progressed) done_cv_.notify_all();
    if (stop_ && queue_.empty() && !busy) return;
    if (!progressed) {
      if (busy)
        cv_.wait_for(g, std::chrono::microseconds(20));
      else
        cv_.wait(g, [&] { return stop_ || !queue_.empty(); });
    }
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
  if (r.ready) (void)hipEventDestroy(r.ready);
  if (out)
    *out = r.blob;
  else if (r.blob)
    isr_blob_free(r.blob);
  if (st) *st = r.st;
  return r.status;
}

}  // namespace isr
