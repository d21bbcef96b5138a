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
  // each slot's stream is created when the slot first takes a request: a
  // context that never serves holds no streams (the device has few hardware
  // queues, and streams created beyond them share queues with other work)
  slots_.resize(n);
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
    if (s.s) (void)hipStreamDestroy(s.s);
  }
  for (auto& kv : reqs_) {
    if (kv.second.blob) isr_blob_free(kv.second.blob);
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    release_copy(kv.second);
  }
}

// A finished (or failed) request no longer reads its copy of the field.
void Scheduler::release_copy(Req& r) {
  if (r.copy) ctx_arena(ctx_)->free(r.copy);
  r.copy = nullptr;
}

int Scheduler::submit(const isr_field* f, uint64_t* req) {
  const long long n = f->order + 1, n3 = n * n * n;
  const size_t fbytes = (size_t)f->ncomp * f->n_elem * n3 * 8, jbytes = f->elem_jac ? (size_t)f->n_elem * 8 : 0;
  const bool copy = (f->flags & ISR_FIELD_COPY) != 0;
  const uint64_t fp = request_footprint(f) + (copy ? fbytes + jbytes + 512 : 0);
  if (fp > ctx_budget(ctx_)) return set_error(ISR_ENOMEM, "request footprint %llu exceeds the HBM budget",
                                              (unsigned long long)fp);
  Req r;
  r.f = *f;
  r.t_submit = now_s();
  std::memset(&r.st, 0, sizeof(r.st));
  hipStream_t ps = (hipStream_t)f->stream;
  if (copy) {
    // copy-on-submit: the field (compact, component after component) and the
    // Jacobians into the arena, on the producer's stream, before returning
    r.copy = ctx_arena(ctx_)->alloc(fbytes + jbytes + 256, true);
    if (!r.copy) return set_error(ISR_ENOMEM, "the copy of the field (%zu bytes) does not fit the HBM budget now", fbytes);
    const size_t stride = (size_t)(f->comp_stride ? f->comp_stride : f->n_elem * n3);
    const size_t cbytes = (size_t)f->n_elem * n3 * 8;
    double* dst = (double*)r.copy;
    bool ok = true;
    for (int c = 0; c < f->ncomp && ok; ++c)
      ok = hipMemcpyAsync((char*)dst + c * cbytes, f->field + c * stride, cbytes, hipMemcpyDeviceToDevice, ps) == hipSuccess;
    double* jac = nullptr;
    if (ok && f->elem_jac) {
      jac = (double*)((char*)r.copy + ((fbytes + 255) & ~size_t(255)));
      ok = hipMemcpyAsync(jac, f->elem_jac, jbytes, hipMemcpyDeviceToDevice, ps) == hipSuccess;
    }
    if (!ok) {
      ctx_arena(ctx_)->free(r.copy);
      return set_error(ISR_EDEVICE, "copy of the field failed: %s", hipGetErrorString(hipGetLastError()));
    }
    r.f.field = dst;
    r.f.comp_stride = 0;
    r.f.elem_jac = jac;
  }
  // the field (or its copy) is ready once the producer's stream reaches this point
  if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r.ready, ps) != hipSuccess) {
    if (r.ready) (void)hipEventDestroy(r.ready);
    if (r.copy) ctx_arena(ctx_)->free(r.copy);
    return set_error(ISR_EDEVICE, "event record on the producer stream failed");
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
  auto start = [&](Slot& s, uint64_t id) {
    if (!s.s && hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking) != hipSuccess) {  // default priority
      s.s = nullptr;
      (void)hipGetLastError();
      return (int)set_error(ISR_EDEVICE, "could not create a stream for a request slot");
    }
    Req& r = reqs_[id];
    (void)hipStreamWaitEvent(s.s, r.ready, 0);
    s.t = Task();
    return task_begin(ctx_, &r.f, s.s, false, &s.t);
  };
  auto end = [&](uint64_t id, int rc) {
    Req& r = reqs_[id];
    r.done = true;
    r.status = rc;
    release_copy(r);
  };
  return admit_fifo(queue_, slots_, ISR_ENOMEM, start, end, &high_);
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
      release_copy(r);
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
