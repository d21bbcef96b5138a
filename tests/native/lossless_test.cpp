// CPU tests of the lossless coder's host entry points (isr_pack_host and
// isr_unpack_host, paper_2407_20731_amd/csrc/isr_lossless.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer: round trips of serialized
// blobs for both codecs, with and without the byte-plane shuffle, and
// corrupt input (truncations, byte flips, forged chunk sizes and headers,
// garbage) that must come back as an error code, never as a crash or an
// out-of-bounds access.  Built by tests/test_arena_admit_cpu.py; prints
// "ALL OK".
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "isr.h"

namespace isr {
// the runtime's error recorder (isr_runtime.cpp is not linked here)
int set_error(int code, const char*, ...) { return code; }
}  // namespace isr

static int g_fail = 0;
#define CHECK(c)                                                                     \
  do {                                                                               \
    if (!(c)) {                                                                      \
      std::fprintf(stderr, "%s:%d: CHECK(%s) failed\n", __FILE__, __LINE__, #c);     \
      ++g_fail;                                                                      \
    }                                                                                \
  } while (0)

typedef std::vector<unsigned char> Bytes;

template <class T>
static void put(Bytes& b, T v) {
  const unsigned char* p = (const unsigned char*)&v;
  b.insert(b.end(), p, p + sizeof(T));
}

// A serialized blob (version-3 layout) with random kept values.
static Bytes make_blob(std::mt19937_64& rng, int ncomp, int64_t ne, int order, int vb) {
  const int n = order + 1, W = (n * n * n + 63) / 64;
  Bytes b = {'I', 'S', 'R', '1'};
  put<uint32_t>(b, 3);
  put<int32_t>(b, order);
  put<int32_t>(b, ncomp);
  put<int64_t>(b, ne);
  put<int32_t>(b, vb);
  put<int32_t>(b, W);
  put<double>(b, 1e-3);
  for (int k = 0; k < 6; ++k) put<int32_t>(b, 0);
  std::vector<uint64_t> kept(ncomp);
  uint64_t voff = 0;
  for (int c = 0; c < ncomp; ++c) {
    kept[c] = rng() % (uint64_t)(ne * 20 + 1);
    for (int k = 0; k < 6; ++k) put<double>(b, 1.0);
    put<uint64_t>(b, kept[c]);
    put<uint64_t>(b, voff);
    put<double>(b, 0.0);
    voff += kept[c];
  }
  for (int64_t i = 0; i < ncomp * ne * W; ++i) put<uint64_t>(b, rng());
  for (int64_t i = 0; i < ncomp * (ne + 1); ++i) put<uint64_t>(b, (uint64_t)i);
  std::normal_distribution<double> g(0.0, 1.0);
  for (uint64_t i = 0; i < voff; ++i) {
    if (vb == 8)
      put<double>(b, g(rng) * 1e-3);
    else
      put<float>(b, (float)(g(rng) * 1e-3));
  }
  return b;
}

static int pack(const Bytes& in, int codec, int level, uint32_t flags, int threads, Bytes& out) {
  uint64_t n = 0;
  int rc = isr_pack_host(in.data(), in.size(), codec, level, flags, threads, nullptr, 0, &n);
  if (rc) return rc;
  out.assign(n, 0);
  return isr_pack_host(in.data(), in.size(), codec, level, flags, threads, out.data(), out.size(), &n);
}

static int unpack(const Bytes& in, Bytes& out) {
  uint64_t n = 0;
  int rc = isr_unpack_host(in.data(), in.size(), nullptr, 0, &n);
  if (rc) return rc;
  if (n > (64ull << 20)) return -100;  // a forged size the test does not allocate
  out.assign(n, 0);
  return isr_unpack_host(in.data(), in.size(), out.data(), out.size(), &n);
}

int main() {
  std::mt19937_64 rng(11);
  // round trips
  const int codecs[][2] = {{ISR_CODEC_ZLIB, 0}, {ISR_CODEC_ZLIB, 1}, {ISR_CODEC_ZLIB, 6}, {ISR_CODEC_BZIP2, 1},
                           {ISR_CODEC_BZIP2, 9}};
  std::vector<Bytes> packs;
  for (auto& cd : codecs)
    for (uint32_t fl : {0u, (uint32_t)ISR_PACK_SHUFFLE})
      for (int vb : {4, 8}) {
        Bytes blob = make_blob(rng, 1 + (int)(rng() % 3), 1 + (int64_t)(rng() % 300), 1 + (int)(rng() % 9), vb);
        Bytes p, back;
        CHECK(pack(blob, cd[0], cd[1], fl, 1 + (int)(rng() % 4), p) == ISR_OK);
        CHECK(unpack(p, back) == ISR_OK && back == blob);
        packs.push_back(p);
      }
  // a blob of several chunks
  {
    Bytes blob = make_blob(rng, 3, 6000, 7, 4);
    Bytes p1, p8, back;
    CHECK(pack(blob, ISR_CODEC_ZLIB, 1, ISR_PACK_SHUFFLE, 1, p1) == ISR_OK);
    CHECK(pack(blob, ISR_CODEC_ZLIB, 1, ISR_PACK_SHUFFLE, 8, p8) == ISR_OK);
    CHECK(p1 == p8 && unpack(p8, back) == ISR_OK && back == blob);
    packs.push_back(p8);
  }
  // refusals of the packer
  {
    Bytes blob = make_blob(rng, 1, 10, 3, 4), p;
    CHECK(pack(blob, ISR_CODEC_ZLIB, 10, 0, 1, p) == ISR_EINVAL);
    CHECK(pack(blob, ISR_CODEC_BZIP2, 0, 0, 1, p) == ISR_EINVAL);
    CHECK(pack(blob, 7, 1, 0, 1, p) == ISR_EINVAL);
    CHECK(pack(blob, ISR_CODEC_ZLIB, 1, 2, 1, p) == ISR_EINVAL);
    Bytes bad = blob;
    std::memcpy(bad.data() + 12, "\xff\xff\xff\x7f", 4);  // ncomp out of range
    CHECK(pack(bad, ISR_CODEC_ZLIB, 1, ISR_PACK_SHUFFLE, 1, p) == ISR_EINVAL);
    bad = blob;
    const int64_t huge = INT64_C(1) << 61;  // element count whose section sizes overflow
    std::memcpy(bad.data() + 16, &huge, 8);
    CHECK(pack(bad, ISR_CODEC_ZLIB, 1, ISR_PACK_SHUFFLE, 1, p) == ISR_EINVAL);
    CHECK(pack(Bytes(10, 0), ISR_CODEC_ZLIB, 1, ISR_PACK_SHUFFLE, 1, p) == ISR_EINVAL);
    uint64_t nb = 0;
    CHECK(isr_pack_host(nullptr, 0, ISR_CODEC_ZLIB, 1, 0, 1, nullptr, 0, &nb) == ISR_EINVAL);
    Bytes one(1, 7), back;
    CHECK(pack(one, ISR_CODEC_BZIP2, 9, 0, 1, p) == ISR_OK && unpack(p, back) == ISR_OK && back == one);
  }
  // corrupt packed input: errors, never crashes
  int rejected = 0, tried = 0;
  for (auto& p : packs) {
    Bytes out;
    for (size_t cut : {(size_t)0, (size_t)3, (size_t)31, (size_t)32, (size_t)40, p.size() / 2, p.size() - 1}) {
      if (cut >= p.size()) continue;
      Bytes t(p.begin(), p.begin() + cut);
      ++tried;
      rejected += unpack(t, out) != ISR_OK;
    }
    for (int k = 0; k < 40; ++k) {
      Bytes t = p;
      t[rng() % t.size()] ^= (unsigned char)(1 + rng() % 255);
      ++tried;
      const int rc = unpack(t, out);
      rejected += rc != ISR_OK;
      if (rc == ISR_OK) {
        uint64_t rn;
        std::memcpy(&rn, t.data() + 16, 8);
        CHECK(out.size() == rn);
      }
    }
    // forged chunk sizes, including ones that overflow an offset sum
    for (uint64_t cs : {(uint64_t)~0ull, (uint64_t)(~0ull - 40), (uint64_t)(1ull << 63), (uint64_t)p.size()}) {
      Bytes t = p;
      std::memcpy(t.data() + 32, &cs, 8);
      CHECK(unpack(t, out) != ISR_OK);
    }
    // forged raw size and chunk count
    Bytes t = p;
    const uint64_t rn = ~0ull;
    std::memcpy(t.data() + 16, &rn, 8);
    CHECK(unpack(t, out) != ISR_OK);
  }
  for (int k = 0; k < 2000; ++k) {
    Bytes g(rng() % 200);
    for (auto& x : g) x = (unsigned char)rng();
    if (g.size() >= 4 && rng() % 2) std::memcpy(g.data(), "ISRZ", 4);
    Bytes out;
    CHECK(unpack(g, out) != ISR_OK || g.size() >= 32);
  }
  std::printf("corrupt inputs: %d of %d rejected\n", rejected, tried);
  CHECK(rejected > tried / 2);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
