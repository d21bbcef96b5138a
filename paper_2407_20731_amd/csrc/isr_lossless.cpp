// Hybrid lossless stage (arXiv 2407.20731, Sec. III-A hybrid approach and
// Sec. IV-B): the lossy step runs on the GPU, synchronously with the
// simulation; its compacted blob is then coded losslessly on separate host
// CPU cores, asynchronously, while the GPU goes on (the paper codes with
// Bzip2 in its NEKO runs and ZLIB in its QE runs, Table II).
//
// Packed format (little endian):
//   "ISRZ", u32 version = 1, u32 codec, u32 flags, u64 raw bytes,
//   u32 chunk count K, u32 raw bytes per chunk (the last may be shorter),
//   K x u64 coded chunk sizes, then the K coded chunks.
// The raw stream is the serialized blob (isr_blob_to_host bytes); with
// ISR_PACK_SHUFFLE its kept values are stored byte plane by byte plane (all
// first bytes, then all second bytes, ...), which groups the slowly varying
// sign and exponent bytes of the floats.  Chunks are coded independently, so
// several host threads code one blob.
#include <hip/hip_runtime.h>
#include <zlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "isr.h"
#include "isr_internal.h"
#include "isr_sched.h"

// libbz2's buffer-to-buffer calls (bzip2 1.0 API; the library ships without
// its header in this image)
extern "C" {
int BZ2_bzBuffToBuffCompress(char* dest, unsigned int* destLen, char* source, unsigned int sourceLen, int blockSize100k,
                             int verbosity, int workFactor);
int BZ2_bzBuffToBuffDecompress(char* dest, unsigned int* destLen, char* source, unsigned int sourceLen, int small,
                               int verbosity);
}

namespace isr {

namespace {

constexpr uint32_t PK_VERSION = 1;
constexpr size_t PK_HDR = 32;
constexpr size_t CHUNK = 4u << 20;  // raw bytes per chunk

struct BlobLayout {
  size_t values_off = 0, values_bytes = 0;
  int vbytes = 0;
  bool ok = false;
};

// Where the kept values sit in a serialized blob (header checked lightly: the
// full check happens when the blob is uploaded).
BlobLayout blob_layout(const unsigned char* p, size_t n) {
  BlobLayout L;
  if (n < 64 || std::memcmp(p, "ISR1", 4) != 0) return L;
  int32_t order, ncomp, vb, W;
  int64_t ne;
  std::memcpy(&order, p + 8, 4);
  std::memcpy(&ncomp, p + 12, 4);
  std::memcpy(&ne, p + 16, 8);
  std::memcpy(&vb, p + 24, 4);
  std::memcpy(&W, p + 28, 4);
  if (ncomp < 1 || ncomp > ISR_MAX_COMP || ne < 1 || (vb != 4 && vb != 8) || W < 1 || W > 64) return L;
  // the bitmap and element offsets alone must fit in n bytes (no overflow below)
  if ((uint64_t)ne > n / (8 * (uint64_t)ncomp * (uint64_t)(W + 1))) return L;
  const size_t off = 64 + 72 * (size_t)ncomp + (size_t)ncomp * ne * W * 8 + (size_t)ncomp * (ne + 1) * 8;
  if (off > n || (n - off) % vb) return L;
  L.values_off = off;
  L.values_bytes = n - off;
  L.vbytes = vb;
  L.ok = true;
  return L;
}

void shuffle(unsigned char* dst, const unsigned char* src, size_t count, int w) {
  for (int b = 0; b < w; ++b)
    for (size_t i = 0; i < count; ++i) dst[b * count + i] = src[i * w + b];
}
void unshuffle(unsigned char* dst, const unsigned char* src, size_t count, int w) {
  for (int b = 0; b < w; ++b)
    for (size_t i = 0; i < count; ++i) dst[i * w + b] = src[b * count + i];
}

size_t code_bound(int codec, size_t n) {
  return codec == ISR_CODEC_ZLIB ? (size_t)compressBound((uLong)n) : n + n / 100 + 600;
}

// Code one chunk; returns the coded size or 0 on failure.
size_t code_chunk(int codec, int level, const unsigned char* src, size_t n, unsigned char* dst, size_t cap) {
  if (codec == ISR_CODEC_ZLIB) {
    uLongf out = (uLongf)cap;
    return compress2(dst, &out, src, (uLong)n, level) == Z_OK ? (size_t)out : 0;
  }
  unsigned int out = (unsigned int)cap;
  return BZ2_bzBuffToBuffCompress((char*)dst, &out, (char*)src, (unsigned int)n, level, 0, 0) == 0 ? (size_t)out : 0;
}

bool decode_chunk(int codec, const unsigned char* src, size_t n, unsigned char* dst, size_t raw) {
  if (codec == ISR_CODEC_ZLIB) {
    uLongf out = (uLongf)raw;
    return uncompress(dst, &out, src, (uLong)n) == Z_OK && out == raw;
  }
  unsigned int out = (unsigned int)raw;
  return BZ2_bzBuffToBuffDecompress((char*)dst, &out, (char*)src, (unsigned int)n, 0, 0) == 0 && out == raw;
}

int check_codec(int codec, int level) {
  if (codec == ISR_CODEC_ZLIB && level >= 0 && level <= 9) return ISR_OK;
  if (codec == ISR_CODEC_BZIP2 && level >= 1 && level <= 9) return ISR_OK;
  return set_error(ISR_EINVAL, "codec %d with level %d is not supported (zlib 0-9, bzip2 1-9)", codec, level);
}

// Code raw (already shuffled if requested) into a packed buffer with up to
// `threads` host threads.
int pack_raw(const std::vector<unsigned char>& raw, int codec, int level, uint32_t flags, int threads,
             std::vector<unsigned char>& out) {
  const size_t n = raw.size();
  const uint32_t K = (uint32_t)std::max<size_t>(1, (n + CHUNK - 1) / CHUNK);
  std::vector<std::vector<unsigned char>> coded(K);
  std::atomic<uint32_t> next{0};
  std::atomic<bool> bad{false};
  auto work = [&]() {
    for (;;) {
      const uint32_t k = next.fetch_add(1);
      if (k >= K) return;
      const size_t o = (size_t)k * CHUNK, len = std::min(CHUNK, n - std::min(n, o));
      coded[k].resize(code_bound(codec, len));
      const size_t got = code_chunk(codec, level, raw.data() + o, len, coded[k].data(), coded[k].size());
      if (!got) bad = true;
      coded[k].resize(got);
    }
  };
  const int nt = std::max(1, std::min<int>(threads, (int)K));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  if (bad) return set_error(ISR_EDEVICE, "lossless coding failed");
  size_t total = PK_HDR + 8 * (size_t)K;
  for (auto& c : coded) total += c.size();
  out.resize(total);
  unsigned char* p = out.data();
  std::memcpy(p, "ISRZ", 4);
  const uint32_t ver = PK_VERSION, cdc = (uint32_t)codec, csz = (uint32_t)CHUNK;
  const uint64_t rn = n;
  std::memcpy(p + 4, &ver, 4);
  std::memcpy(p + 8, &cdc, 4);
  std::memcpy(p + 12, &flags, 4);
  std::memcpy(p + 16, &rn, 8);
  std::memcpy(p + 24, &K, 4);
  std::memcpy(p + 28, &csz, 4);
  size_t at = PK_HDR + 8 * (size_t)K;
  for (uint32_t k = 0; k < K; ++k) {
    const uint64_t cs = coded[k].size();
    std::memcpy(p + PK_HDR + 8 * (size_t)k, &cs, 8);
    std::memcpy(p + at, coded[k].data(), cs);
    at += cs;
  }
  return ISR_OK;
}

// The raw stream of a serialized blob: the blob itself, with its values
// section shuffled under ISR_PACK_SHUFFLE.
int raw_of(const unsigned char* blob, size_t n, uint32_t flags, std::vector<unsigned char>& raw) {
  raw.assign(blob, blob + n);
  if (flags & ISR_PACK_SHUFFLE) {
    const BlobLayout L = blob_layout(blob, n);
    if (!L.ok) return set_error(ISR_EINVAL, "not a serialized ISR1 blob");
    shuffle(raw.data() + L.values_off, blob + L.values_off, L.values_bytes / L.vbytes, L.vbytes);
  }
  return ISR_OK;
}

int host_threads_default() {
  const unsigned h = std::thread::hardware_concurrency();
  return h ? (int)std::min(h, 12u) : 12;
}

}  // namespace

// ---- asynchronous packing on the context's host threads ----------------------
// One dispatcher thread per context takes jobs in order: it waits for the
// job's device-to-host copy (enqueued on the packer's own stream at submit),
// then codes the blob with the context's host threads.
struct Packer {
  struct Job {
    uint64_t id = 0;
    int codec = 0, level = 0;
    uint32_t flags = 0;
    std::vector<unsigned char> ser;   // the serialized blob's header
    unsigned char* pinned = nullptr;  // device body lands here
    size_t body = 0, hb = 0, staged = 0;  // staged: size of the pinned buffer
    hipEvent_t copied = nullptr;
    bool done = false;
    int status = 0;
    double t_submit = 0, t_done = 0;
    std::vector<unsigned char> out;
  };
  int device = 0, threads = 12;
  hipStream_t s = nullptr;
  // pinned staging buffers, reused across jobs (pinning host memory costs
  // milliseconds; a submit should not): free ones by size
  std::multimap<size_t, unsigned char*> staging;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;

  // a pinned buffer of at least n bytes (under mu)
  unsigned char* take(size_t n, size_t* got) {
    auto it = staging.lower_bound(n);
    if (it != staging.end()) {
      unsigned char* p = it->second;
      *got = it->first;
      staging.erase(it);
      return p;
    }
    const size_t want = std::max<size_t>((n + (1u << 20) - 1) & ~size_t((1u << 20) - 1), 1u << 20);
    unsigned char* p = nullptr;
    if (hipHostMalloc((void**)&p, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    *got = want;
    return p;
  }
  // return a buffer (under mu); at most 8 are kept
  void give_back(unsigned char* p, size_t n) {
    if (!p) return;
    staging.emplace(n, p);
    while (staging.size() > 8) {
      (void)hipHostFree(staging.begin()->second);
      staging.erase(staging.begin());
    }
  }
  static double now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
  }
  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> g(mu);
    for (;;) {
      cv.wait(g, [&] { return stop || !queue.empty(); });
      if (queue.empty()) return;  // stop requested and nothing left
      Job* j = jobs[queue.front()].get();
      queue.pop_front();
      g.unlock();
      // wait for the blob's copy by polling: a blocking wait here would sit
      // inside the runtime beside the submitting thread's launches
      int rc = ISR_OK;
      for (;;) {
        const hipError_t q = hipEventQuery(j->copied);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) {
          rc = ISR_EDEVICE;
          break;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
      std::vector<unsigned char> raw, out;
      if (rc == ISR_OK) {
        // the serialized blob: header (taken at submit) and the copied body
        std::vector<unsigned char> ser(j->hb + j->body);
        std::memcpy(ser.data(), j->ser.data(), j->hb);
        std::memcpy(ser.data() + j->hb, j->pinned, j->body);
        rc = raw_of(ser.data(), ser.size(), j->flags, raw);
      }
      if (rc == ISR_OK) rc = pack_raw(raw, j->codec, j->level, j->flags, threads, out);
      g.lock();
      (void)hipEventDestroy(j->copied);
      give_back(j->pinned, j->staged);
      j->pinned = nullptr;
      j->ser.clear();
      j->ser.shrink_to_fit();
      j->out.swap(out);
      j->status = rc;
      j->t_done = now();
      j->done = true;
      done_cv.notify_all();
    }
  }
  ~Packer() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
    for (auto& kv : jobs) {
      if (kv.second->pinned) (void)hipHostFree(kv.second->pinned);
    }
    for (auto& kv : staging) (void)hipHostFree(kv.second);
    if (s) (void)hipStreamDestroy(s);
  }
};

Packer* packer_create(int device, int threads) {
  std::unique_ptr<Packer> p(new Packer());
  p->device = device;
  p->threads = threads > 0 ? threads : host_threads_default();
  // the copy stream is created at the first submit: a context that never
  // packs holds none (the device has few hardware queues to share)
  Packer* raw = p.get();
  p->worker = std::thread([raw] { raw->loop(); });
  return p.release();
}

void packer_destroy(Packer* p) { delete p; }

int packer_submit(Packer* p, const unsigned char* hdr, size_t hb, const void* dev_body, size_t body, int codec,
                  int level, uint32_t flags, uint64_t* job) {
  std::unique_ptr<Packer::Job> j(new Packer::Job());
  j->codec = codec;
  j->level = level;
  j->flags = flags;
  j->hb = hb;
  j->body = body;
  j->t_submit = Packer::now();
  j->ser.assign(hdr, hdr + hb);  // the header only: the body is assembled by the packer's thread
  {
    std::lock_guard<std::mutex> g(p->mu);
    if (!p->s && hipStreamCreateWithFlags(&p->s, hipStreamNonBlocking) != hipSuccess) {  // default priority
      p->s = nullptr;
      (void)hipGetLastError();
      return set_error(ISR_EDEVICE, "could not create the lossless stage's copy stream");
    }
    j->pinned = p->take(body, &j->staged);
  }
  if (!j->pinned) return set_error(ISR_ENOMEM, "pinned staging of %zu bytes failed", body);
  if (hipEventCreateWithFlags(&j->copied, hipEventDisableTiming) != hipSuccess ||
      hipMemcpyAsync(j->pinned, dev_body, body, hipMemcpyDeviceToHost, p->s) != hipSuccess ||
      hipEventRecord(j->copied, p->s) != hipSuccess) {
    (void)hipStreamSynchronize(p->s);
    std::lock_guard<std::mutex> g(p->mu);
    p->give_back(j->pinned, j->staged);
    if (j->copied) (void)hipEventDestroy(j->copied);
    return set_error(ISR_EDEVICE, "copy of the blob to the host failed");
  }
  {
    std::lock_guard<std::mutex> g(p->mu);
    j->id = p->next_id++;
    *job = j->id;
    p->queue.push_back(j->id);
    p->jobs.emplace(j->id, std::move(j));
  }
  p->cv.notify_one();
  return ISR_OK;
}

int packer_poll(Packer* p, uint64_t job, int wait_ms, void* out, uint64_t cap, uint64_t* out_bytes, double* secs) {
  std::unique_lock<std::mutex> g(p->mu);
  auto it = p->jobs.find(job);
  if (it == p->jobs.end()) return set_error(ISR_ENOTFOUND, "unknown packing job %llu", (unsigned long long)job);
  Packer::Job* j = it->second.get();
  if (!j->done) {
    if (wait_ms < 0)
      p->done_cv.wait(g, [&] { return j->done; });
    else if (wait_ms > 0)
      p->done_cv.wait_for(g, std::chrono::milliseconds(wait_ms), [&] { return j->done; });
    if (!j->done) return ISR_PENDING;
  }
  if (j->status != ISR_OK) {
    const int rc = j->status;
    p->jobs.erase(it);
    return rc;
  }
  if (out_bytes) *out_bytes = j->out.size();
  if (secs) *secs = j->t_done - j->t_submit;
  if (!out) return ISR_OK;  // size query: the job stays
  if (cap < j->out.size())
    return set_error(ISR_EINVAL, "buffer of %llu bytes is smaller than the packed blob (%zu)", (unsigned long long)cap,
                     j->out.size());
  std::memcpy(out, j->out.data(), j->out.size());
  p->jobs.erase(it);
  return ISR_OK;
}

}  // namespace isr

extern "C" {

static int pack_host(const void* blob, uint64_t n, int32_t codec, int32_t level, uint32_t flags, int32_t threads,
                     void* out, uint64_t cap, uint64_t* out_bytes) {
  using namespace isr;
  if (!blob || !out_bytes) return set_error(ISR_EINVAL, "blob or out_bytes is NULL");
  int rc = check_codec(codec, level);
  if (rc) return rc;
  if (flags & ~(uint32_t)ISR_PACK_SHUFFLE) return set_error(ISR_EINVAL, "unknown packing flags 0x%x", flags);
  std::vector<unsigned char> raw, packed;
  rc = raw_of((const unsigned char*)blob, n, flags, raw);
  if (rc) return rc;
  rc = pack_raw(raw, codec, level, flags, threads > 0 ? threads : host_threads_default(), packed);
  if (rc) return rc;
  *out_bytes = packed.size();
  if (!out) return ISR_OK;
  if (cap < packed.size())
    return set_error(ISR_EINVAL, "buffer of %llu bytes is smaller than the packed blob (%zu)", (unsigned long long)cap,
                     packed.size());
  std::memcpy(out, packed.data(), packed.size());
  return ISR_OK;
}

static int unpack_host(const void* packed, uint64_t n, void* out, uint64_t cap, uint64_t* out_bytes) {
  using namespace isr;
  if (!packed || !out_bytes) return set_error(ISR_EINVAL, "packed or out_bytes is NULL");
  const unsigned char* p = (const unsigned char*)packed;
  if (n < PK_HDR || std::memcmp(p, "ISRZ", 4) != 0) return set_error(ISR_EINVAL, "not an ISRZ packed blob");
  uint32_t ver, codec, flags, K, csz;
  uint64_t raw_n;
  std::memcpy(&ver, p + 4, 4);
  std::memcpy(&codec, p + 8, 4);
  std::memcpy(&flags, p + 12, 4);
  std::memcpy(&raw_n, p + 16, 8);
  std::memcpy(&K, p + 24, 4);
  std::memcpy(&csz, p + 28, 4);
  if (ver != PK_VERSION || (codec != ISR_CODEC_ZLIB && codec != ISR_CODEC_BZIP2) || csz == 0 ||
      (uint64_t)K != std::max<uint64_t>(1, (raw_n + csz - 1) / csz) || n < PK_HDR + 8 * (uint64_t)K)
    return set_error(ISR_EINVAL, "corrupt ISRZ header");
  *out_bytes = raw_n;
  if (!out) return ISR_OK;
  if (cap < raw_n) return set_error(ISR_EINVAL, "buffer of %llu bytes is smaller than the blob (%llu)",
                                    (unsigned long long)cap, (unsigned long long)raw_n);
  std::vector<unsigned char> raw(raw_n);
  uint64_t at = PK_HDR + 8 * (uint64_t)K;
  for (uint32_t k = 0; k < K; ++k) {
    uint64_t cs;
    std::memcpy(&cs, p + PK_HDR + 8 * (size_t)k, 8);
    const uint64_t o = (uint64_t)k * csz, len = std::min<uint64_t>(csz, raw_n - o);
    if (cs > n - at || !decode_chunk((int)codec, p + at, cs, raw.data() + o, len))
      return set_error(ISR_EINVAL, "corrupt ISRZ chunk %u", k);
    at += cs;
  }
  if (at != n) return set_error(ISR_EINVAL, "ISRZ size does not match its chunks");
  unsigned char* dst = (unsigned char*)out;
  std::memcpy(dst, raw.data(), raw_n);
  if (flags & ISR_PACK_SHUFFLE) {
    const BlobLayout L = blob_layout(raw.data(), raw_n);
    if (!L.ok) return set_error(ISR_EINVAL, "unpacked bytes are not an ISR1 blob");
    unshuffle(dst + L.values_off, raw.data() + L.values_off, L.values_bytes / L.vbytes, L.vbytes);
  }
  return ISR_OK;
}

// No C++ exception crosses the C ABI (allocation or thread creation failures
// become error codes).
int isr_pack_host(const void* blob, uint64_t n, int32_t codec, int32_t level, uint32_t flags, int32_t threads,
                  void* out, uint64_t cap, uint64_t* out_bytes) {
  try {
    return pack_host(blob, n, codec, level, flags, threads, out, cap, out_bytes);
  } catch (const std::bad_alloc&) {
    return isr::set_error(ISR_ENOMEM, "host memory exhausted while packing");
  } catch (...) {
    return isr::set_error(ISR_EDEVICE, "packing failed on the host");
  }
}

int isr_unpack_host(const void* packed, uint64_t n, void* out, uint64_t cap, uint64_t* out_bytes) {
  try {
    return unpack_host(packed, n, out, cap, out_bytes);
  } catch (const std::bad_alloc&) {
    return isr::set_error(ISR_ENOMEM, "host memory exhausted while unpacking");
  } catch (...) {
    return isr::set_error(ISR_EDEVICE, "unpacking failed on the host");
  }
}

}  // extern "C"
