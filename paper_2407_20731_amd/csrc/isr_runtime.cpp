// Host runtime behind the C ABI (include/isr.h): contexts, the HBM arena,
// the compression pipeline, blobs, decompression and the request queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <string>
#include <thread>
#include <vector>

#include "isr.h"
#include "isr_internal.h"
#include "isr_sched.h"

using namespace isr;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace isr {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace isr

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(ISR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// arena: device sub-allocator over large hipMalloc chunks, capped by a budget

namespace isr {

// chunks of the arena come straight from the device allocator
static void* dev_chunk_alloc(size_t bytes, void*) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

static void dev_chunk_free(void* p, void*) { (void)hipFree(p); }

}  // namespace isr

// ---------------------------------------------------------------------------
// context and blob

struct isr_blob {
  isr_ctx* ctx = nullptr;
  void* dev = nullptr;  // [voff area 256 B][bitmap][elem_ptr][values]
  size_t dev_bytes = 0;
  int order = 0, ncomp = 0, vbytes = 8, W = 0, precision = 0, status = 0;
  int engine = 0, tile = 0;  // FP32 / BF16: the engine (and dense tile) whose inverse decompresses it
  int value_kind = 0;        // 0: coefficient values; 1: quantisation codes (integers held by FP32)
  int64_t n_elem = 0;
  double tol = 0;
  struct Hdr {
    double U2, B, tau, dropped, err2, rel;
    uint64_t kept, voff;
    double qstep;  // quantisation step of the codes (value_kind 1), else 0
  } comp[ISR_MAX_COMP];
  uint64_t total_kept = 0;
  u64* voff() const { return (u64*)dev; }
  double* qstep_dev() const { return (double*)((char*)dev + 64); }  // device copy of the steps
  u64* bitmap() const { return (u64*)((char*)dev + 256); }
  size_t bitmap_bytes() const { return (size_t)ncomp * n_elem * W * 8; }
  u64* elem_ptr() const { return (u64*)((char*)bitmap() + bitmap_bytes()); }
  size_t ptr_bytes() const { return (size_t)ncomp * (n_elem + 1) * 8; }
  void* values() const { return (char*)elem_ptr() + ptr_bytes(); }
  size_t values_bytes() const { return (size_t)total_kept * vbytes; }
  static constexpr size_t HDR = 64, CHDR = 72;
  size_t serialized() const { return HDR + CHDR * ncomp + bitmap_bytes() + ptr_bytes() + values_bytes(); }
};

struct isr_ctx {
  int device = 0;
  uint32_t flags = 0;
  int num_cu = 256;
  std::unique_ptr<isr::Arena> arena;
  void* tables_dev = nullptr;
  DevTables tab[ISR_MAX_ORDER + 1];
  std::mutex mu;  // serialises device pipelines
  std::unique_ptr<isr::Scheduler> sched;
  isr::Packer* packer = nullptr;  // hybrid lossless stage on host threads
  int max_inflight = 8;
  std::atomic<int> tile[ISR_MAX_ORDER + 1][3];  // tile shape per (order, precision); -1 = built-in
  std::string tune_path;           // tile table file (read at create, written by the autotuner)
  CompState* st_host = nullptr;  // pinned state copy of isr_compress_noalloc (under mu)
  std::mutex host_mu;            // pools of pinned per-request state buffers and completion events
  std::vector<CompState*> host_all, host_free;
  std::unordered_map<CompState*, CompState*> host_dev;  // device address of each state buffer (null: none)
  std::vector<hipEvent_t> ev_all, ev_free;
};

static int set_device(isr_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return ISR_OK;
}

static int upload_tables(isr_ctx* c) {
  // one allocation: per order A, V, w3, g3 (FP64) then A32, V32 (FP32)
  std::vector<char> host;
  size_t offs[ISR_MAX_ORDER + 1][6];
  for (int N = 1; N <= ISR_MAX_ORDER; ++N) {
    HostTables t;
    if (!host_tables(N, &t)) return fail(ISR_EINVAL, "table generation failed for order %d", N);
    const int n = N + 1, n2 = n * n, n3 = n2 * n;
    auto put = [&](const void* src, size_t bytes) {
      size_t o = (host.size() + 255) & ~size_t(255);
      host.resize(o + bytes);
      std::memcpy(host.data() + o, src, bytes);
      return o;
    };
    offs[N][0] = put(t.A, n2 * 8);
    offs[N][1] = put(t.V, n2 * 8);
    offs[N][2] = put(t.w3, n3 * 8);
    offs[N][3] = put(t.g3, n3 * 8);
    float a32[256], v32[256];
    for (int k = 0; k < n2; ++k) {
      a32[k] = (float)t.A[k];
      v32[k] = (float)t.V[k];
    }
    offs[N][4] = put(a32, n2 * 4);
    offs[N][5] = put(v32, n2 * 4);
  }
  HIPCHK(hipMalloc(&c->tables_dev, host.size()));
  HIPCHK(hipMemcpy(c->tables_dev, host.data(), host.size(), hipMemcpyHostToDevice));
  char* base = (char*)c->tables_dev;
  for (int N = 1; N <= ISR_MAX_ORDER; ++N) {
    c->tab[N].A = (const double*)(base + offs[N][0]);
    c->tab[N].V = (const double*)(base + offs[N][1]);
    c->tab[N].w3 = (const double*)(base + offs[N][2]);
    c->tab[N].g3 = (const double*)(base + offs[N][3]);
    c->tab[N].A32 = (const float*)(base + offs[N][4]);
    c->tab[N].V32 = (const float*)(base + offs[N][5]);
  }
  return ISR_OK;
}

// ---------------------------------------------------------------------------
// argument checks and sizes

static int check_field(const isr_field* f) {
  if (!f) return fail(ISR_EINVAL, "field descriptor is NULL");
  if (!f->field) return fail(ISR_EINVAL, "field pointer is NULL");
  if (((uintptr_t)f->field) & 7) return fail(ISR_EINVAL, "field pointer is not 8-byte aligned");
  if (f->elem_jac && (((uintptr_t)f->elem_jac) & 7)) return fail(ISR_EINVAL, "elem_jac is not 8-byte aligned");
  if (f->order < 1 || f->order > ISR_MAX_ORDER) return fail(ISR_EINVAL, "order %d outside [1, %d]", f->order, ISR_MAX_ORDER);
  if (f->ncomp < 1 || f->ncomp > ISR_MAX_COMP) return fail(ISR_EINVAL, "ncomp %d outside [1, %d]", f->ncomp, ISR_MAX_COMP);
  if (f->n_elem < 1) return fail(ISR_EINVAL, "n_elem must be >= 1");
  const long long n = f->order + 1, n3 = n * n * n;
  if ((unsigned long long)f->n_elem * n3 >= (1ull << 32)) return fail(ISR_EINVAL, "n_elem * (order+1)^3 must be < 2^32");
  if (std::isnan(f->tol)) return fail(ISR_EINVAL, "tol is NaN");
  if (f->precision != ISR_PREC_FP64 && f->precision != ISR_PREC_FP32 && f->precision != ISR_PREC_BF16)
    return fail(ISR_EINVAL, "unknown precision %d", f->precision);
  if (f->comp_stride < 0 || (f->comp_stride > 0 && f->comp_stride < f->n_elem * n3))
    return fail(ISR_EINVAL, "comp_stride smaller than one component");
  if (f->flags & ~ISR_FIELD_COPY) return fail(ISR_EINVAL, "unknown field flags 0x%x", f->flags);
  return ISR_OK;
}

namespace isr {

Sizes plan_sizes(const isr_field* f, int tile, bool full_lists) {
  Sizes z;
  const long long n = f->order + 1, n3 = n * n * n;
  const int nc = f->ncomp;
  z.nv = (u64)f->n_elem * n3;
  z.W = words_per_elem(f->order);
  z.tiles = tiles_per_comp(f->order, f->n_elem);
  z.vbytes = f->precision == ISR_PREC_FP64 ? 8 : 4;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o += (b + 255) & ~size_t(255);
    return r;
  };
  z.off_histE = take((size_t)nc * HBINS * sizeof(HistBin));
  z.off_histN = take((size_t)nc * HBINS * sizeof(HistBin));
  z.off_histR = take((size_t)nc * HBINS * sizeof(HistBin));
  z.off_histL = take((size_t)(NLEV - 1) * nc * RBINS * sizeof(HistBin));
  z.off_histEs = take((size_t)nc * HBINS * sizeof(HistBin));
  z.off_histNs = take((size_t)nc * HBINS * sizeof(HistBin));
  // a 1/32 sample of the tiles predicts the boundary bin when there are enough tiles
  z.sample_stride = z.tiles >= 1024 ? 32 : 0;
  z.off_st = take((size_t)nc * sizeof(CompState));
  z.off_ticket = take(256);
  z.off_lookback = take((size_t)nc * z.tiles * 8);
  z.off_done = take(16 * 8 * sizeof(u32));
  z.zero_bytes = o;
  z.list_cap = full_lists || z.nv <= (1ull << 20) ? z.nv : std::max<u64>(z.nv / 8, 1ull << 20);
  z.off_lists = take((size_t)nc * 2 * z.list_cap * 8);  // list 0, then lists 1 and 2 at half size
  z.fast = fast_order(f->order, f->precision);
  z.tile = z.fast && f->precision != ISR_PREC_FP64 && dense_shape(f->order, tile) ? tile : 0;
  if (z.fast) {
    const long long epw = fast_epw(f->order, z.tile), ftiles = (f->n_elem + epw - 1) / epw;
    z.sample_stride = std::max<long long>(1, ftiles / 1024);  // about 1024 sampled tiles
    z.off_lidx = take((size_t)nc * z.list_cap * 4);
    z.off_cnt = take((size_t)nc * f->n_elem * 4);
    z.off_slotsA = take((size_t)nc * FAST_GMAX * 8 * 8);
    z.off_slotsB = take((size_t)nc * FAST_GMAX * 4 * 8);
    z.off_chunk = take((size_t)nc * ((f->n_elem + 1023) / 1024) * 8);
  }
  z.scratch_bytes = o;
  z.blob_max = 256 + (size_t)nc * f->n_elem * z.W * 8 + (size_t)nc * (f->n_elem + 1) * 8 + (size_t)nc * z.nv * z.vbytes;
  return z;
}

}  // namespace isr

// Device addresses of a blob's sections (per-component value offsets, bitmaps,
// offset tables, values).
struct BlobPtrs {
  u64* voff;
  u64* bitmap;
  u64* elem_ptr;
  void* values;
};

static BlobPtrs blob_ptrs(const isr_blob* b) { return {b->voff(), b->bitmap(), b->elem_ptr(), b->values()}; }

// Record which engine's inverse reproduces the reconstruction that pass B
// measured (FP32 / BF16 blobs; FP64 blobs always use the fixed-order FP64
// inverse): the streaming path's wave-tile / large-order engine (tile 0) or
// dense-tile engine, else the general passes.
static void set_engine(isr_blob* b, bool fast, int tile) {
  b->engine = b->precision == ISR_PREC_FP64 || !fast ? ENG_GENERAL : (tile > 0 ? ENG_DENSE : ENG_WAVE);
  b->tile = b->engine == ENG_DENSE ? tile : 0;
}

static Job make_job(isr_ctx* c, const isr_field* f, const Sizes& z, char* scratch, const BlobPtrs& bp) {
  Job j;
  std::memset(&j, 0, sizeof(j));
  const long long n = f->order + 1, n3 = n * n * n;
  j.u = f->field;
  j.jac = f->elem_jac;
  j.comp_stride = f->comp_stride ? f->comp_stride : f->n_elem * n3;
  j.n_elem = f->n_elem;
  j.order = f->order;
  j.ncomp = f->ncomp;
  j.precision = f->precision;
  j.vbytes = z.vbytes;
  j.tol = f->tol;
  j.cut_scale = 1.0;
  for (int k = 0; k < 8; ++k) j.Bov[k] = -1.0;
  j.tab = c->tab[f->order];
  j.histE = (HistBin*)(scratch + z.off_histE);
  j.histN = (HistBin*)(scratch + z.off_histN);
  j.histR = (HistBin*)(scratch + z.off_histR);
  j.histL = (HistBin*)(scratch + z.off_histL);
  j.histEs = (HistBin*)(scratch + z.off_histEs);
  j.histNs = (HistBin*)(scratch + z.off_histNs);
  j.sample_stride = z.sample_stride;
  j.st = (CompState*)(scratch + z.off_st);
  j.ticket = (u32*)(scratch + z.off_ticket);
  j.lookback = (u64*)(scratch + z.off_lookback);
  j.lists = (u64*)(scratch + z.off_lists);
  j.list_cap = z.list_cap;
  j.done = (u32*)(scratch + z.off_done);
  j.tile = z.tile;
  if (z.fast) {
    j.lidx = (u32*)(scratch + z.off_lidx);
    j.cnt = (u32*)(scratch + z.off_cnt);
    j.slotsA = (long long*)(scratch + z.off_slotsA);
    j.slotsB = (long long*)(scratch + z.off_slotsB);
    j.chunk = (u64*)(scratch + z.off_chunk);
    j.nchunk = (f->n_elem + 1023) / 1024;
  }
  j.bitmap = bp.bitmap;
  j.elem_ptr = bp.elem_ptr;
  j.values = bp.values;
  j.voff = bp.voff;
  return j;
}

// Enqueue every phase of one compression on stream s (no host sync).
namespace isr {

// Streaming path (isr_engine.cuh): sample, pass A, exact window bins and
// level-1 selection, refinement, per-element counts and offsets, pass B with
// the finalize step.  A threshold outside the sampled window sets ST_MISS in
// the selection; every later kernel then returns at once and the host runs
// the general pipeline.
// Grids of the streaming path's phases for job j (workgroups per component),
// and the passes' grids and extraction headroom stored in j.  The persistent
// batch launch uses the same values, so a snapshot's results do not depend on
// how it was launched.
struct FastGrids {
  int gs, gl, rgx, gsc;  // sample, list passes (gather, count), refinement levels, offset scans
};

static FastGrids fast_setup(isr_ctx* c, Job& j, const Sizes& z) {
  const int nc = j.ncomp, prec = j.precision;
  const long long epw = fast_epw(j.order, j.tile);
  const long long ftiles = (j.n_elem + epw - 1) / epw;
  auto grid = [&](int kind) {
    const long long slots = (long long)c->num_cu * resident_fast(kind, prec, j.order, j.tile);
    long long g = std::max<long long>(1, slots / nc);
    g = std::min<long long>(g, (ftiles + 3) / 4);
    return (int)std::max<long long>(1, std::min<long long>(g, FAST_GMAX));
  };
  j.gA = grid(F_PASSA);
  j.gB = grid(F_PASSB);
  // terms per lane: values per lane per tile times tiles per wave
  const long long per_wave = (ftiles + 4ll * std::min(j.gA, j.gB) - 1) / (4ll * std::min(j.gA, j.gB));
  const long long terms = fast_lane_terms(j.order, j.tile) * per_wave;
  int h = 1;
  while ((1ll << (h - 1)) < terms) ++h;
  j.xh = std::max(7, std::min(20, h));
  FastGrids g;
  const long long ss = j.sample_stride > 0 ? j.sample_stride : 1;
  const long long stiles = (ftiles + ss - 1) / ss;
  // sixteen sampled tiles per workgroup; one per wavefront at N >= 8, whose
  // tiles are large (1000+ values): there the serial chain of tiles per
  // wavefront costs more than the extra workgroups' histogram atomics
  g.gs = (int)std::max<long long>(1, j.order >= 8 ? std::min<long long>(256, (stiles + 3) / 4)
                                                  : std::min<long long>(64, (stiles + 15) / 16));
  // list passes over ~2 % of the values; few refinement workgroups (each
  // flushes up to RBINS sub-bins with global atomics: 32 per component beat
  // 16 and 64 at 100M values)
  g.gl = (int)std::max<long long>(1, std::min<long long>(GATHER_GMAX, (long long)(z.nv >> 17) + 1));
  g.rgx = std::max(1, std::min(32, (int)(z.nv >> 20) + 1));
  g.gsc = scan_grid_elems(j.n_elem);
  return g;
}

// Streaming path: sample, pass A, exact window bins and level-1 selection,
// refinement, per-element counts and offsets, pass B with the finalize step.
// A threshold outside the sampled window sets ST_MISS in the selection; every
// later kernel then returns at once and the host runs the general pipeline.
static int enqueue_fast(isr_ctx* c, const Job& j0, const Sizes& z, hipStream_t s, hipEvent_t* ev) {
  Job j = j0;
  const int prec = j.precision;
  const FastGrids g = fast_setup(c, j, z);
  auto rec = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], s);
  };
  rec(7);
  HIPCHK(launch_zero((void*)j.histE, z.zero_bytes, s));
  HIPCHK(launch_fast(F_SAMPLE, prec, j, g.gs, s));
  HIPCHK(launch_fast_tail(F_SAMPLE, j, s));
  rec(0);
  HIPCHK(launch_fast(F_PASSA, prec, j, j.gA, s));
  rec(1);
  HIPCHK(launch_gather(j, g.gl, s));
  rec(2);
  rec(3);
  HIPCHK(launch_refsel(j, g.rgx, s));
  HIPCHK(launch_count(j, g.gl, s));
  rec(4);
  HIPCHK(launch_fast(F_PASSB, prec, j, j.gB, s));
  rec(5);
  HIPCHK(launch_fast_tail(F_PASSB, j, s));
  rec(6);
  return ISR_OK;
}

int enqueue_pipeline(isr_ctx* c, const Job& j, const Sizes& z, hipStream_t s, hipEvent_t* ev, bool fast) {
  if (fast) return enqueue_fast(c, j, z, s, ev);
  const int nc = j.ncomp;
  const long long tiles = z.tiles;
  const int prec = j.precision;
  const int nn = j.order + 1, tile_vals = (256 / (nn * nn) > 0 ? 256 / (nn * nn) : 1) * nn * nn * nn;
  // persistent grids sized to what is resident at once
  auto grid_per_comp = [&](int kind) {
    const long long slots = (long long)c->num_cu * resident_blocks(kind, prec, j.order);
    long long gx = std::min<long long>(tiles, std::max<long long>(1, slots / nc));
    // each workgroup may add at most 2^21 - 1 values to one LDS bin
    const long long min_gx = (tiles * (long long)tile_vals + (1ll << 21) - 2) / ((1ll << 21) - 1);
    return (int)std::max<long long>(gx, std::min<long long>(tiles, min_gx));
  };
  auto rec = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], s);
  };
  rec(7);
  HIPCHK(launch_zero((void*)j.histE, z.zero_bytes, s));
  if (j.sample_stride > 0) {
    const long long stiles = (tiles + j.sample_stride - 1) / j.sample_stride;
    const long long slots = (long long)c->num_cu * resident_blocks(K_PASS1, prec, j.order);
    const int sgx = (int)std::min<long long>(stiles, std::max<long long>(1, slots / nc));
    HIPCHK(launch_pass(K_PASS1, prec, j, sgx, s, nullptr, 1));
    HIPCHK(launch_select1(j, 1, s));
  }
  rec(0);
  HIPCHK(launch_pass(K_PASS1, prec, j, grid_per_comp(K_PASS1), s, nullptr, 0));
  rec(1);
  HIPCHK(launch_select1(j, 0, s));
  rec(2);
  HIPCHK(launch_pass(K_PASS2, prec, j, grid_per_comp(K_PASS2), s));
  rec(3);
  const int rgx = std::max(1, std::min(64, (int)(z.nv >> 20) + 1));
  HIPCHK(launch_refsel(j, rgx, s));
  rec(4);
  const long long slots3 = (long long)c->num_cu * resident_blocks(K_PASS3, prec, j.order);
  const int g3 = (int)std::min<long long>(tiles * nc, slots3);
  HIPCHK(launch_pass(K_PASS3, prec, j, g3, s));
  rec(5);
  HIPCHK(launch_finalize(j, s));
  rec(6);
  return ISR_OK;
}

}  // namespace isr

static int status_from_flags(int flags) {
  if (flags & ST_NONFINITE) return fail(ISR_EINVAL, "field holds a non-finite value");
  if (flags & ST_OVERFLOW) return fail(ISR_EINVAL, "an energy overflowed FP64 (field magnitude too large)");
  if (flags & (ST_SPIN | ST_LIST)) return fail(ISR_EDEVICE, "internal selection error (flags 0x%x)", flags);
  return ISR_OK;
}

static isr_blob* new_blob(isr_ctx* c, const isr_field* f, const Sizes& z) {
  isr_blob* b = new isr_blob();
  b->ctx = c;
  b->order = f->order;
  b->ncomp = f->ncomp;
  b->n_elem = f->n_elem;
  b->vbytes = z.vbytes;
  b->W = z.W;
  b->tol = f->tol;
  b->precision = f->precision;
  b->dev_bytes = z.blob_max;
  b->dev = c->arena->alloc(z.blob_max, true);
  if (!b->dev) {
    delete b;
    return nullptr;
  }
  return b;
}

static void fill_stats(isr_blob* b, const CompState* hs, isr_stats* st) {
  for (int k = 0; k < b->ncomp; ++k) {
    auto& h = b->comp[k];
    h.U2 = hs[k].U2;
    h.B = hs[k].B;
    h.tau = hs[k].tau;
    h.dropped = hs[k].dropped;
    h.err2 = hs[k].err2;
    h.rel = hs[k].rel;
    h.kept = hs[k].kept;
  }
  uint64_t vo = 0;
  for (int k = 0; k < b->ncomp; ++k) {
    b->comp[k].voff = vo;
    vo += b->comp[k].kept;
  }
  b->total_kept = vo;
  if (st) {
    for (int k = 0; k < b->ncomp; ++k) {
      st->norm2[k] = b->comp[k].U2;
      st->budget[k] = b->comp[k].B;
      st->tau[k] = b->comp[k].tau;
      st->dropped[k] = b->comp[k].dropped;
      st->err2[k] = b->comp[k].err2;
      st->rel_err[k] = b->comp[k].rel;
      st->kept[k] = b->comp[k].kept;
    }
    const long long n = b->order + 1;
    st->in_bytes = (uint64_t)b->ncomp * b->n_elem * n * n * n * 8;
    st->blob_bytes = b->serialized();
    st->cr = st->in_bytes ? (double)((int64_t)st->in_bytes - (int64_t)st->blob_bytes) / (double)st->in_bytes : 0.0;
    st->precision = b->precision;
  }
}

namespace isr {

int ctx_device(const isr_ctx* c) { return c->device; }
Arena* ctx_arena(isr_ctx* c) { return c->arena.get(); }
int ctx_max_inflight(const isr_ctx* c) { return c->max_inflight; }
uint64_t ctx_budget(const isr_ctx* c) { return c->arena->budget(); }

int ctx_tile(const isr_ctx* c, int order, int precision) {
  if (precision < ISR_PREC_FP32 || precision > ISR_PREC_BF16 || order < 1 || order > ISR_MAX_ORDER) return 0;
  const int t = c->tile[order][precision].load();
  return t >= 0 ? t : default_tile(order, precision);
}

// Footprint a request needs from the arena (scratch + worst-case blob).
uint64_t request_footprint(const isr_field* f) {
  Sizes z = plan_sizes(f, 0, false);
  return (uint64_t)z.scratch_bytes + z.blob_max + 512;
}

static CompState* grab_host_state(isr_ctx* c) {
  std::lock_guard<std::mutex> g(c->host_mu);
  if (c->host_free.empty()) {
    CompState* p = nullptr;
    if (hipHostMalloc((void**)&p, sizeof(CompState) * ISR_MAX_COMP, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    c->host_all.push_back(p);
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipGetLastError();
      d = nullptr;
    }
    c->host_dev[p] = (CompState*)d;
    return p;
  }
  CompState* p = c->host_free.back();
  c->host_free.pop_back();
  return p;
}

static void put_host_state(isr_ctx* c, CompState* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(c->host_mu);
  c->host_free.push_back(p);
}

static CompState* host_state_dev(isr_ctx* c, CompState* p) {
  std::lock_guard<std::mutex> g(c->host_mu);
  auto it = c->host_dev.find(p);
  return it == c->host_dev.end() ? nullptr : it->second;
}

// Completion events are reused across requests (creating one per request
// costs host time between back-to-back requests).
static hipEvent_t grab_event(isr_ctx* c) {
  std::lock_guard<std::mutex> g(c->host_mu);
  if (c->ev_free.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    c->ev_all.push_back(e);
    return e;
  }
  hipEvent_t e = c->ev_free.back();
  c->ev_free.pop_back();
  return e;
}

static void put_event(isr_ctx* c, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> g(c->host_mu);
  c->ev_free.push_back(e);
}

static int task_enqueue(Task* t) {
  Job j = t->j;
  if (!t->fast) j.hs_out = nullptr;  // the streaming path's last kernel writes the state itself
  int rc = enqueue_pipeline(t->c, j, t->z, t->s, t->timing ? t->ev : nullptr, t->fast);
  if (rc) return rc;
  if (!j.hs_out) HIPCHK(launch_state_out(t->j.st, t->hs, t->f.ncomp, t->s));
  HIPCHK(hipEventRecord(t->done, t->s));
  return ISR_OK;
}

void task_release(Task* t) {
  if (t->scratch) t->c->arena->free(t->scratch);
  t->scratch = nullptr;
  if (t->b) {
    t->c->arena->free(t->b->dev);
    delete t->b;
    t->b = nullptr;
  }
  put_event(t->c, t->done);
  t->done = nullptr;
  if (t->timing)
    for (auto& e : t->ev) (void)hipEventDestroy(e);
  t->timing = false;
  put_host_state(t->c, t->hs);
  t->hs = nullptr;
}

// Rounding repair after a finished pass: for every component whose measured
// error exceeds tol, lower its budget to B (tol/rel)^2 (1 - 2^-20); keep the
// others' budgets (which reproduces their results).  At most 4 repairs.
// Returns whether another pass is needed.
static bool plan_repair(const isr_field* f, const CompState* hs, int iters, double* Bov) {
  bool again = false;
  if (f->tol >= 0.0 && iters < 4) {
    for (int k = 0; k < f->ncomp; ++k) {
      if (hs[k].rel > f->tol) {
        const double fr = f->tol / hs[k].rel;
        Bov[k] = (hs[k].B * (fr * fr)) * (1.0 - 0x1p-20);
        again = true;
      } else {
        Bov[k] = hs[k].B;  // unchanged, reproduces the same result
      }
    }
  }
  return again;
}

// Validate, allocate and enqueue the whole pipeline on stream s.  ISR_ENOMEM
// when the request does not fit the HBM budget right now.
int task_begin(isr_ctx* c, const isr_field* f, hipStream_t s, bool timing, Task* t) {
  int rc = check_field(f);
  if (rc) return rc;
  t->c = c;
  t->f = *f;
  t->s = s;
  t->t_start = now_s();
  t->z = plan_sizes(f, ctx_tile(c, f->order, f->precision), t->full_lists);
  t->scratch = (char*)c->arena->alloc(t->z.scratch_bytes);
  if (!t->scratch) return fail(ISR_ENOMEM, "scratch of %zu bytes does not fit the HBM budget", t->z.scratch_bytes);
  t->b = new_blob(c, f, t->z);
  if (!t->b) {
    c->arena->free(t->scratch);
    t->scratch = nullptr;
    return fail(ISR_ENOMEM, "blob of %zu bytes does not fit the HBM budget", t->z.blob_max);
  }
  t->hs = grab_host_state(c);
  if (!t->hs || !(t->done = grab_event(c))) {
    task_release(t);
    return fail(ISR_EDEVICE, "could not create host state or event");
  }
  t->j = make_job(c, f, t->z, t->scratch, blob_ptrs(t->b));
  t->j.cut_scale = t->cut_scale;
  t->j.hs_out = host_state_dev(c, t->hs);
  t->fast = t->z.fast;
  t->timing = timing;
  if (timing)
    for (auto& e : t->ev) (void)hipEventCreate(&e);
  std::memset(&t->st, 0, sizeof(t->st));
  rc = task_enqueue(t);
  if (rc) task_release(t);
  return rc;
}

// After t->done completed: check the result, repair (ISR_PENDING: enqueued
// again) or finish (final status; the blob moves to *out on OK / ETOL).
int task_step(Task* t, isr_blob** out) {
  CompState* hs = t->hs;
  const isr_field* f = &t->f;
  int flags = 0;
  for (int k = 0; k < f->ncomp; ++k) flags |= hs[k].flags;
  if (t->fast && (flags & ST_MISS)) {
    // the threshold fell outside the sampled window: run the general pipeline
    // (no sample window this time), keeping any budget override
    if (t->timing) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t->ev[7], t->ev[6]) == hipSuccess) t->st.phase_ms[7] += ms;
    }
    t->fast = false;
    t->j.sample_stride = 0;
    int rc = task_enqueue(t);
    if (rc) {
      task_release(t);
      return rc;
    }
    return ISR_PENDING;
  }
  if ((flags & ST_LIST) && !t->full_lists) {
    // a candidate list outgrew its first-attempt capacity (energies bunched
    // in a few exponent bins): the same attempt again with lists for every
    // value, keeping the path and any budget override
    double Bov[8];
    std::memcpy(Bov, t->j.Bov, sizeof(Bov));
    const long long ss = t->j.sample_stride;
    CompState* const hs_out = t->j.hs_out;
    t->full_lists = true;
    t->c->arena->free(t->scratch);
    t->z = plan_sizes(f, t->z.tile, true);
    t->scratch = (char*)t->c->arena->alloc(t->z.scratch_bytes);
    if (!t->scratch) {
      task_release(t);
      return fail(ISR_ENOMEM, "candidate lists for every value (%zu bytes of scratch) do not fit the HBM budget",
                  t->z.scratch_bytes);
    }
    t->j = make_job(t->c, f, t->z, t->scratch, blob_ptrs(t->b));
    t->j.cut_scale = t->cut_scale;
    t->j.sample_stride = ss;
    t->j.hs_out = hs_out;
    std::memcpy(t->j.Bov, Bov, sizeof(Bov));
    int rc = task_enqueue(t);
    if (rc) {
      task_release(t);
      return rc;
    }
    return ISR_PENDING;
  }
  int rc = status_from_flags(flags);
  if (rc) {
    task_release(t);
    return rc;
  }
  if (t->timing) {
    // phases 0..5 between events 0..6; phase 8 (zero fill, sample pass and
    // window selection) from event 7 to event 0
    float ms[9] = {};
    for (int k = 0; k < 6; ++k) (void)hipEventElapsedTime(&ms[k], t->ev[k], t->ev[k + 1]);
    (void)hipEventElapsedTime(&ms[8], t->ev[7], t->ev[0]);
    for (int k : {0, 1, 2, 3, 4, 5, 8}) {
      if (t->iters == 0)
        t->st.phase_ms[k] = ms[k];
      else
        t->repair_ms += ms[k];
    }
  }
  // rounding repair: lower B where the measured error exceeds tol
  const bool again = plan_repair(f, hs, t->iters, t->j.Bov);
  if (again) {
    ++t->iters;
    rc = task_enqueue(t);
    if (rc) {
      task_release(t);
      return rc;
    }
    return ISR_PENDING;
  }
  isr_blob* b = t->b;
  fill_stats(b, hs, &t->st);
  bool within = true;
  if (f->tol >= 0.0)
    for (int k = 0; k < f->ncomp; ++k) within = within && !(hs[k].rel > f->tol);
  b->status = within ? ISR_OK : ISR_ETOL;
  // return the unused tail of the worst-case value reservation; under a tight
  // budget move the blob to an exact-size allocation instead (a shrunk
  // reservation leaves a gap that the next scratch may not fit)
  const size_t used = 256 + b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
  bool moved = false;
  if (used < b->dev_bytes / 2 && t->c->arena->budget() < 8 * (t->z.scratch_bytes + t->z.blob_max)) {
    t->c->arena->free(t->scratch);
    t->scratch = nullptr;
    void* q = t->c->arena->alloc(used, true);
    if (q && hipMemcpyAsync(q, b->dev, used, hipMemcpyDeviceToDevice, t->s) == hipSuccess &&
        hipStreamSynchronize(t->s) == hipSuccess) {
      t->c->arena->free(b->dev);
      b->dev = q;
      moved = true;
    } else {
      (void)hipGetLastError();
      if (q) t->c->arena->free(q);
    }
  }
  if (!moved) t->c->arena->shrink(b->dev, used);
  b->dev_bytes = (used + 255) & ~size_t(255);
  t->st.phase_ms[6] = t->repair_ms;
  t->st.repair_iters = t->iters;
  t->st.path = t->fast ? 1 : 0;
  set_engine(b, t->fast, t->z.tile);
  t->st.status = b->status;
  t->st.t_start = t->t_start;
  t->st.t_done = now_s();
  t->b = nullptr;  // handed over
  task_release(t);
  *out = b;
  if (!within) fail(ISR_ETOL, "relative error above tol after %d repairs", t->iters);
  return b->status;
}

// Several snapshots of orders 5, 7 and 9 in ONE persistent launch
// (isr_batch.cuh); other batches run one after another.
// Snapshots the persistent kernel does not take run through the request
// scheduler: up to max_inflight at once on their own streams, so that one
// snapshot's latency-bound selection kernels overlap another's streaming
// passes.  Every result equals the snapshot compressed alone.
static int run_batch_concurrent(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st) {
  std::vector<uint64_t> ids(count, 0);
  std::vector<int> sub(count, ISR_OK);
  // largest snapshots first: the last ones to start are short, so the
  // streams drain together instead of one large pipeline running alone
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto work = [&](int i) {
    const long long n = fs[i].order + 1;
    return (long long)fs[i].n_elem * n * n * n * fs[i].ncomp;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  for (int i : order) sub[i] = c->sched->submit(&fs[i], &ids[i]);
  int first = ISR_OK;
  for (int i = 0; i < count; ++i) {
    outs[i] = nullptr;
    int rc = sub[i];
    if (rc == ISR_OK) rc = c->sched->poll(ids[i], -1, &outs[i], st ? &st[i] : nullptr);
    if (st) st[i].status = rc;
    if (rc != ISR_OK && first == ISR_OK) first = rc;
  }
  return first;
}

// FP32 / BF16 batch of orders 5, 7, 9 (each with the tile shape the
// persistent kernel holds): one persistent launch of the streaming path
// (isr_fbatch.cuh).  A snapshot whose threshold fell outside its sampled
// window, or whose error needs a rounding repair, is then compressed alone,
// which is what it would have got alone as well.
static int run_batch_stream(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st) {
  const int prec = fs[0].precision;
  hipStream_t s = (hipStream_t)fs[0].stream;
  const double t_start = now_s();
  struct Snap {
    Sizes z;
    char* scratch = nullptr;
    isr_blob* b = nullptr;
    Job j;
    FastGrids g;
    CompState* hs = nullptr;
  };
  std::vector<Snap> sn(count);
  auto cleanup = [&]() {
    for (auto& x : sn) {
      if (x.scratch) c->arena->free(x.scratch);
      if (x.b) {
        c->arena->free(x.b->dev);
        delete x.b;
      }
      put_host_state(c, x.hs);
      x = Snap();
    }
  };
  for (int i = 0; i < count; ++i) {
    outs[i] = nullptr;
    Snap& x = sn[i];
    x.z = plan_sizes(&fs[i], ctx_tile(c, fs[i].order, fs[i].precision));
    x.scratch = (char*)c->arena->alloc(x.z.scratch_bytes);
    x.b = x.scratch ? new_blob(c, &fs[i], x.z) : nullptr;
    x.hs = grab_host_state(c);
    if (!x.scratch || !x.b || !x.hs) {
      cleanup();
      return fail(ISR_ENOMEM, "batch of %d snapshots does not fit the HBM budget", count);
    }
    x.j = make_job(c, &fs[i], x.z, x.scratch, blob_ptrs(x.b));
    x.g = fast_setup(c, x.j, x.z);
  }
  // pairs of the largest snapshots first in every phase: their passes start
  // first, so their selection chains are ready when the queue reaches them and
  // few workgroups spin on unfinished dependencies
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sn[a].z.nv > sn[b].z.nv; });
  std::vector<int> psnap, pcomp;
  for (int i : order)
    for (int cc = 0; cc < fs[i].ncomp; ++cc) {
      psnap.push_back(i);
      pcomp.push_back(cc);
    }
  const int np = (int)psnap.size();
  std::vector<long long> items((size_t)NFQ * (np + 1), 0);
  BatchCtl B;
  std::memset(&B, 0, sizeof(B));
  B.npairs = np;
  long long off = 0;
  for (int ph = 0; ph < NFQ; ++ph) {
    B.phase_off[ph] = off;
    long long* row = &items[(size_t)ph * (np + 1)];
    row[0] = 0;
    for (int q = 0; q < np; ++q) {
      const Snap& x = sn[psnap[q]];
      long long cnt = 1;
      if (ph == FQ_SAMPLE)
        cnt = x.g.gs;
      else if (ph == FQ_PASSA)
        cnt = x.j.gA;
      else if (ph == FQ_PASSB)
        cnt = x.j.gB;
      else if (ph == FQ_GATHER || ph == FQ_COUNT)
        cnt = x.g.gl;
      else if (ph == FQ_SCAN1 || ph == FQ_SCAN2)
        cnt = x.g.gsc;
      else
        cnt = x.g.rgx;
      row[q + 1] = row[q] + cnt;
    }
    off += row[np];
  }
  B.phase_off[NFQ] = off;
  const size_t sz_jobs = sizeof(Job) * count, sz_pairs = sizeof(int) * np, sz_items = sizeof(long long) * items.size(),
               sz_done = sizeof(u32) * NFQ * np;
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t o_jobs = 0, o_ps = al(sz_jobs), o_pc = o_ps + al(sz_pairs), o_items = o_pc + al(sz_pairs),
               o_done = o_items + al(sz_items), o_ticket = o_done + al(sz_done), o_err = o_ticket + 256,
               total = o_err + 256;
  char* tab = (char*)c->arena->alloc(total);
  if (!tab) {
    cleanup();
    return fail(ISR_ENOMEM, "batch tables do not fit the HBM budget");
  }
  std::vector<char> host(total, 0);
  for (int i = 0; i < count; ++i) std::memcpy(host.data() + o_jobs + sizeof(Job) * i, &sn[i].j, sizeof(Job));
  std::memcpy(host.data() + o_ps, psnap.data(), sz_pairs);
  std::memcpy(host.data() + o_pc, pcomp.data(), sz_pairs);
  std::memcpy(host.data() + o_items, items.data(), sz_items);
  B.jobs = (const Job*)(tab + o_jobs);
  B.pair_snap = (const int*)(tab + o_ps);
  B.pair_comp = (const int*)(tab + o_pc);
  B.items = (const long long*)(tab + o_items);
  B.done = (u32*)(tab + o_done);
  B.ticket = (unsigned long long*)(tab + o_ticket);
  B.err = (int*)(tab + o_err);
  int rc = ISR_OK;
  int err_host = 0;
  do {
    for (int i = 1; i < count; ++i) {
      if (fs[i].stream == fs[0].stream) continue;
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
        (void)hipEventRecord(e, (hipStream_t)fs[i].stream);
        (void)hipStreamWaitEvent(s, e, 0);
        (void)hipEventDestroy(e);
      }
    }
    if (hipMemcpyAsync(tab, host.data(), total, hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch table upload failed");
      break;
    }
    for (int i = 0; i < count && !rc; ++i)
      if (launch_zero(sn[i].scratch, sn[i].z.zero_bytes, s) != hipSuccess) rc = fail(ISR_EDEVICE, "zero fill failed");
    if (rc) break;
    // LDS for the largest of the shapes this batch holds (and the
    // order-independent phases)
    size_t lds = fbatch_lds(prec, 0, 0);
    for (int i = 0; i < count; ++i) lds = std::max(lds, fbatch_lds(prec, fs[i].order, sn[i].z.tile));
    const int grid = c->num_cu * fbatch_resident(prec, lds);
    if (launch_fbatch(prec, B, grid, lds, s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch launch failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    for (int i = 0; i < count; ++i)
      (void)launch_state_out(sn[i].j.st, sn[i].hs, fs[i].ncomp, s);
    (void)hipMemcpyAsync(&err_host, B.err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if (err_host) rc = fail(ISR_EDEVICE, "batch: a bounded wait expired");
  } while (0);
  c->arena->free(tab);
  if (rc) {
    cleanup();
    return rc;
  }
  int first = ISR_OK;
  for (int i = 0; i < count; ++i) {
    Snap& x = sn[i];
    const isr_field* f = &fs[i];
    int flags = 0;
    bool again = false;
    for (int k = 0; k < f->ncomp; ++k) {
      flags |= x.hs[k].flags;
      if (f->tol >= 0.0 && x.hs[k].rel > f->tol) again = true;
    }
    if (flags & ST_MISS) again = true;
    isr_stats* sti = st ? &st[i] : nullptr;
    int r = (flags & ST_MISS) ? ISR_OK : status_from_flags(flags);
    if (r == ISR_OK && again) {
      c->arena->free(x.scratch);
      x.scratch = nullptr;
      c->arena->free(x.b->dev);
      delete x.b;
      x.b = nullptr;
      r = run_compress(c, f, &outs[i], sti);
    } else if (r == ISR_OK) {
      isr_blob* b = x.b;
      isr_stats tmp;
      std::memset(&tmp, 0, sizeof(tmp));
      fill_stats(b, x.hs, &tmp);
      b->status = ISR_OK;
      const size_t used = 256 + b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
      c->arena->shrink(b->dev, used);
      b->dev_bytes = (used + 255) & ~size_t(255);
      tmp.status = ISR_OK;
      tmp.path = 2;
      set_engine(b, true, x.z.tile);
      tmp.t_start = t_start;
      tmp.t_done = now_s();
      if (sti) *sti = tmp;
      outs[i] = b;
      x.b = nullptr;
    }
    if (sti) sti->status = r;
    if (r != ISR_OK && first == ISR_OK) first = r;
  }
  cleanup();
  return first;
}

int run_batch(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st) {
  if (count <= 0) return ISR_OK;
  bool persistent = true, stream = true;
  for (int i = 0; i < count; ++i) {
    const int o = fs[i].order, p = fs[i].precision;
    if ((o != 5 && o != 7 && o != 9) || p != fs[0].precision) persistent = stream = false;
    // FP64: the persistent kernel of the general passes (exact, so equal to
    // compressing alone); FP32 / BF16: the persistent kernel of the streaming
    // passes, with each order's tile shape from the context's table (built-in
    // or autotuned; the kernel holds every candidate), or on request the
    // concurrent per-snapshot pipelines
    if (p != ISR_PREC_FP64) persistent = false;
    if (p == ISR_PREC_FP64 || !stream || !fbatch_shape(o, ctx_tile(c, o, p))) stream = false;
  }
  // The persistent streaming launch is opt-in: every queue item publishes its
  // results to later phases through device-scope release/acquire counters,
  // and on gfx950 each such fence writes back and invalidates an XCD's L2;
  // over tens of thousands of items that costs more than the per-snapshot
  // launches it saves (measured: 32 snapshots, 26.8 GB, BF16: 61 ms in one
  // persistent launch, 27 ms as stream pipelines).  A handful of snapshots
  // also keeps the phases of one snapshot apart in the queue.
  if (stream && count >= FBATCH_MIN && (c->flags & ISR_FLAG_BATCH_PERSISTENT))
    return run_batch_stream(c, fs, count, outs, st);
  if (!persistent) return run_batch_concurrent(c, fs, count, outs, st);
  const int prec = fs[0].precision;
  hipStream_t s = (hipStream_t)fs[0].stream;
  const double t_start = now_s();
  struct Snap {
    Sizes z;
    char* scratch = nullptr;
    isr_blob* b = nullptr;
    Job j;
    CompState* hs = nullptr;
  };
  std::vector<Snap> sn(count);
  auto cleanup = [&]() {
    for (auto& x : sn) {
      if (x.scratch) c->arena->free(x.scratch);
      if (x.b) {
        c->arena->free(x.b->dev);
        delete x.b;
      }
      put_host_state(c, x.hs);
      x = Snap();
    }
  };
  for (int i = 0; i < count; ++i) {
    outs[i] = nullptr;
    Snap& x = sn[i];
    x.z = plan_sizes(&fs[i], 0);
    x.z.sample_stride = x.z.tiles >= 1024 ? 32 : 0;  // the batch kernel runs the general passes
    x.scratch = (char*)c->arena->alloc(x.z.scratch_bytes);
    x.b = x.scratch ? new_blob(c, &fs[i], x.z) : nullptr;
    x.hs = grab_host_state(c);
    if (!x.scratch || !x.b || !x.hs) {
      cleanup();
      return fail(ISR_ENOMEM, "batch of %d snapshots does not fit the HBM budget", count);
    }
    x.j = make_job(c, &fs[i], x.z, x.scratch, blob_ptrs(x.b));
  }
  // pairs and items of every phase
  std::vector<int> psnap, pcomp;
  for (int i = 0; i < count; ++i)
    for (int cc = 0; cc < fs[i].ncomp; ++cc) {
      psnap.push_back(i);
      pcomp.push_back(cc);
    }
  const int np = (int)psnap.size();
  std::vector<long long> items((size_t)NPH * (np + 1), 0);
  BatchCtl B;
  std::memset(&B, 0, sizeof(B));
  B.npairs = np;
  long long off = 0;
  for (int ph = 0; ph < NPH; ++ph) {
    B.phase_off[ph] = off;
    long long* row = &items[(size_t)ph * (np + 1)];
    row[0] = 0;
    for (int q = 0; q < np; ++q) {
      const Snap& x = sn[psnap[q]];
      const long long tiles = x.z.tiles;
      const long long k1 = std::min<long long>(std::max<long long>(1, (tiles + 31) / 32), 4096);
      long long cnt = 1;
      if (ph == PH_P0) {
        const long long st_tiles = x.z.sample_stride ? (tiles + x.z.sample_stride - 1) / x.z.sample_stride : 0;
        cnt = x.z.sample_stride ? std::max<long long>(1, std::min<long long>(st_tiles, (st_tiles + 7) / 8)) : 0;
      } else if (ph == PH_P1 || ph == PH_P2) {
        cnt = k1;
      } else if (ph == PH_R2 || ph == PH_R3 || ph == PH_R4 || ph == PH_R5 || ph == PH_R6) {
        cnt = std::min<long long>(64, std::max<long long>(1, (long long)(x.z.nv / 262144)));
      } else if (ph == PH_P3) {
        cnt = tiles;
      }
      row[q + 1] = row[q] + cnt;
    }
    off += row[np];
  }
  B.phase_off[NPH] = off;
  // device tables: jobs, pair maps, item prefixes, counters
  const size_t sz_jobs = sizeof(Job) * count, sz_pairs = sizeof(int) * np, sz_items = sizeof(long long) * items.size(),
               sz_done = sizeof(u32) * NPH * np;
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t o_jobs = 0, o_ps = al(sz_jobs), o_pc = o_ps + al(sz_pairs), o_items = o_pc + al(sz_pairs),
               o_done = o_items + al(sz_items), o_ticket = o_done + al(sz_done), o_err = o_ticket + 256,
               total = o_err + 256;
  char* tab = (char*)c->arena->alloc(total);
  if (!tab) {
    cleanup();
    return fail(ISR_ENOMEM, "batch tables do not fit the HBM budget");
  }
  std::vector<char> host(total, 0);
  for (int i = 0; i < count; ++i) std::memcpy(host.data() + o_jobs + sizeof(Job) * i, &sn[i].j, sizeof(Job));
  std::memcpy(host.data() + o_ps, psnap.data(), sz_pairs);
  std::memcpy(host.data() + o_pc, pcomp.data(), sz_pairs);
  std::memcpy(host.data() + o_items, items.data(), sz_items);
  B.jobs = (const Job*)(tab + o_jobs);
  B.pair_snap = (const int*)(tab + o_ps);
  B.pair_comp = (const int*)(tab + o_pc);
  B.items = (const long long*)(tab + o_items);
  B.done = (u32*)(tab + o_done);
  B.ticket = (unsigned long long*)(tab + o_ticket);
  B.err = (int*)(tab + o_err);
  int rc = ISR_OK;
  int err_host = 0;
  do {
    // the fields of the other snapshots must be ready on their own streams
    for (int i = 1; i < count; ++i) {
      if (fs[i].stream == fs[0].stream) continue;
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
        (void)hipEventRecord(e, (hipStream_t)fs[i].stream);
        (void)hipStreamWaitEvent(s, e, 0);
        (void)hipEventDestroy(e);
      }
    }
    if (hipMemcpyAsync(tab, host.data(), total, hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch table upload failed");
      break;
    }
    for (int i = 0; i < count && !rc; ++i)
      if (launch_zero(sn[i].scratch, sn[i].z.zero_bytes, s) != hipSuccess) rc = fail(ISR_EDEVICE, "zero fill failed");
    if (rc) break;
    const size_t lds = batch_lds(prec);
    const int grid = c->num_cu * batch_resident(prec, lds);
    if (launch_batch(prec, B, grid, lds, s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch launch failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    for (int i = 0; i < count; ++i)
      (void)launch_state_out(sn[i].j.st, sn[i].hs, fs[i].ncomp, s);
    (void)hipMemcpyAsync(&err_host, B.err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "batch failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if (err_host) rc = fail(ISR_EDEVICE, "batch: a bounded wait expired");
  } while (0);
  c->arena->free(tab);
  if (rc) {
    cleanup();
    return rc;
  }
  int first = ISR_OK;
  for (int i = 0; i < count; ++i) {
    Snap& x = sn[i];
    const isr_field* f = &fs[i];
    int flags = 0;
    bool repair = false;
    for (int k = 0; k < f->ncomp; ++k) {
      flags |= x.hs[k].flags;
      if (f->tol >= 0.0 && x.hs[k].rel > f->tol) repair = true;
    }
    int r = status_from_flags(flags);
    isr_stats* sti = st ? &st[i] : nullptr;
    if (r == ISR_OK && repair) {
      // rounding left the error above tol: the single path repairs it
      c->arena->free(x.scratch);
      x.scratch = nullptr;
      c->arena->free(x.b->dev);
      delete x.b;
      x.b = nullptr;
      r = run_compress(c, f, &outs[i], sti);
    } else if (r == ISR_OK) {
      isr_blob* b = x.b;
      isr_stats tmp;
      std::memset(&tmp, 0, sizeof(tmp));
      fill_stats(b, x.hs, &tmp);
      b->status = ISR_OK;
      const size_t used = 256 + b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
      c->arena->shrink(b->dev, used);
      b->dev_bytes = (used + 255) & ~size_t(255);
      tmp.status = ISR_OK;
      tmp.t_start = t_start;
      tmp.t_done = now_s();
      if (sti) *sti = tmp;
      outs[i] = b;
      x.b = nullptr;
    }
    if (sti) sti->status = r;
    if (r != ISR_OK && first == ISR_OK) first = r;
  }
  cleanup();
  return first;
}

// Run one compression to completion on the caller's stream.
int run_compress(isr_ctx* c, const isr_field* f, isr_blob** out, isr_stats* st, double cut_scale) {
  *out = nullptr;
  Task t;
  t.cut_scale = cut_scale;
  int rc = task_begin(c, f, (hipStream_t)f->stream, (c->flags & ISR_FLAG_TIMING) && st, &t);
  if (rc) return rc;
  for (;;) {
    if (hipEventSynchronize(t.done) != hipSuccess) {
      rc = fail(ISR_EDEVICE, "device pipeline failed: %s", hipGetErrorString(hipGetLastError()));
      task_release(&t);
      return rc;
    }
    rc = task_step(&t, out);
    if (rc != ISR_PENDING) break;
  }
  if (st) *st = t.st;
  return rc;
}

}  // namespace isr

// Tile-shape table file: one "order precision tile" line per tuned entry.
static void read_tile_table(isr_ctx* c) {
  FILE* fp = std::fopen(c->tune_path.c_str(), "r");
  if (!fp) return;  // not written yet
  int o, p, t;
  while (std::fscanf(fp, "%d %d %d", &o, &p, &t) == 3)
    if (o >= 1 && o <= ISR_MAX_ORDER && p >= ISR_PREC_FP32 && p <= ISR_PREC_BF16 && fast_order(o, p) &&
        (t == 0 || dense_shape(o, t)))
      c->tile[o][p] = t;
  std::fclose(fp);
}

static int write_tile_table(isr_ctx* c) {
  const std::string tmp = c->tune_path + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return fail(ISR_EINVAL, "cannot write the tile table %s", tmp.c_str());
  for (int o = 1; o <= ISR_MAX_ORDER; ++o)
    for (int p = ISR_PREC_FP32; p <= ISR_PREC_BF16; ++p)
      if (c->tile[o][p].load() >= 0) std::fprintf(fp, "%d %d %d\n", o, p, c->tile[o][p].load());
  const bool ok = std::fclose(fp) == 0 && std::rename(tmp.c_str(), c->tune_path.c_str()) == 0;
  return ok ? ISR_OK : fail(ISR_EINVAL, "cannot write the tile table %s", c->tune_path.c_str());
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* isr_version(void) { return "isr 0.1 (gfx950)"; }

const char* isr_last_error(void) { return g_err.c_str(); }

int isr_create(const isr_config* cfg, isr_ctx** out) {
  if (!out) return fail(ISR_EINVAL, "out is NULL");
  *out = nullptr;
  isr_config d;
  std::memset(&d, 0, sizeof(d));
  if (cfg) d = *cfg;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (d.device < 0 || d.device >= ndev) return fail(ISR_EINVAL, "device %d not present (%d devices)", d.device, ndev);
  std::unique_ptr<isr_ctx> c(new isr_ctx());
  c->device = d.device;
  c->flags = d.flags;
  c->max_inflight = d.max_inflight > 0 ? d.max_inflight : 8;
  HIPCHK(hipSetDevice(c->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, c->device));
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->arena.reset(new isr::Arena(d.hbm_budget_bytes ? d.hbm_budget_bytes : (64ull << 30), isr::dev_chunk_alloc,
                                isr::dev_chunk_free, nullptr));
  for (auto& row : c->tile)
    for (auto& t : row) t = -1;
  if (d.autotune_path) {
    c->tune_path = d.autotune_path;
    read_tile_table(c.get());
  }
  int rc = upload_tables(c.get());
  if (rc) return rc;
  HIPCHK(hipHostMalloc((void**)&c->st_host, sizeof(CompState) * ISR_MAX_COMP, hipHostMallocMapped | hipHostMallocCoherent));
  rc = isr::noalloc_init(c->device);  // address of the allocation-free entry point's scratch on this GPU
  if (rc) return rc;
  c->sched.reset(new isr::Scheduler(c.get()));
  c->packer = isr::packer_create(c->device, d.host_threads);
  if (!c->packer) return fail(ISR_EDEVICE, "could not create the lossless packer");
  *out = c.release();
  return ISR_OK;
}

int isr_destroy(isr_ctx* c) {
  if (!c) return fail(ISR_EINVAL, "ctx is NULL");
  (void)hipSetDevice(c->device);
  c->sched.reset();
  isr::packer_destroy(c->packer);
  c->packer = nullptr;
  (void)hipDeviceSynchronize();
  c->arena.reset();
  if (c->tables_dev) (void)hipFree(c->tables_dev);
  if (c->st_host) (void)hipHostFree(c->st_host);
  for (CompState* p : c->host_all) (void)hipHostFree(p);
  for (hipEvent_t e : c->ev_all) (void)hipEventDestroy(e);
  delete c;
  return ISR_OK;
}

int isr_compress(isr_ctx* c, const isr_field* f, isr_blob** out, isr_stats* st) {
  if (!c || !out) return fail(ISR_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  if (st) std::memset(st, 0, sizeof(*st));
  int rc = set_device(c);
  if (rc) return rc;
  const double t0 = now_s();
  std::lock_guard<std::mutex> g(c->mu);
  rc = run_compress(c, f, out, st);
  if (st) st->t_submit = t0;
  return rc;
}

int isr_compress_batch(isr_ctx* c, const isr_field* fs, int32_t count, isr_blob** outs, isr_stats* st) {
  if (!c || !fs || !outs || count < 0) return fail(ISR_EINVAL, "bad batch arguments");
  int rc = set_device(c);
  if (rc) return rc;
  for (int i = 0; i < count; ++i) {
    outs[i] = nullptr;
    int r = check_field(&fs[i]);
    if (r) return r;
  }
  std::lock_guard<std::mutex> g(c->mu);
  return isr::run_batch(c, fs, count, outs, st);
}

int isr_get_tile(isr_ctx* c, int32_t order, int32_t precision, int32_t* tile) {
  if (!c || !tile) return fail(ISR_EINVAL, "ctx or tile is NULL");
  if (order < 1 || order > ISR_MAX_ORDER || precision < ISR_PREC_FP64 || precision > ISR_PREC_BF16)
    return fail(ISR_EINVAL, "bad order %d or precision %d", order, precision);
  *tile = ctx_tile(c, order, precision);
  return ISR_OK;
}

int isr_set_tile(isr_ctx* c, int32_t order, int32_t precision, int32_t tile) {
  if (!c) return fail(ISR_EINVAL, "ctx is NULL");
  if (precision != ISR_PREC_FP32 && precision != ISR_PREC_BF16)
    return fail(ISR_EINVAL, "tile shapes exist for FP32 and BF16 only");
  if (order < 1 || order > ISR_MAX_ORDER || !fast_order(order, precision))
    return fail(ISR_EINVAL, "order %d has no streaming path", order);
  if (tile != -1 && tile != 0 && !dense_shape(order, tile))
    return fail(ISR_EINVAL, "tile shape %d is not compiled for order %d", tile, order);
  c->tile[order][precision] = tile;
  return ISR_OK;
}

int isr_autotune(isr_ctx* c, const isr_field* f, int32_t reps, isr_tune_report* rep) {
  if (!c) return fail(ISR_EINVAL, "ctx is NULL");
  int rc = check_field(f);
  if (rc) return rc;
  if (f->precision == ISR_PREC_FP64 || !fast_order(f->order, f->precision))
    return fail(ISR_EINVAL, "nothing to tune for order %d precision %d", f->order, f->precision);
  rc = set_device(c);
  if (rc) return rc;
  int cand[16];
  const int nc = tile_candidates(f->order, cand, 16);
  const int before = c->tile[f->order][f->precision].load();
  double best_ms = 0.0;
  int best = -1;
  isr_tune_report r;
  std::memset(&r, 0, sizeof(r));
  for (int k = 0; k < nc; ++k) {
    c->tile[f->order][f->precision] = cand[k];
    double ms = 0.0;
    for (int it = 0; it <= std::max(1, (int)reps); ++it) {
      isr_blob* b = nullptr;
      const double t0 = now_s();
      {
        std::lock_guard<std::mutex> g(c->mu);
        rc = run_compress(c, f, &b, nullptr);
      }
      const double dt = (now_s() - t0) * 1e3;
      if (b) isr_blob_free(b);
      if (rc != ISR_OK && rc != ISR_ETOL) {
        c->tile[f->order][f->precision] = before;
        return rc;
      }
      if (it > 0) ms = it == 1 ? dt : std::min(ms, dt);  // the first call warms up
    }
    r.tile[k] = cand[k];
    r.ms[k] = ms;
    if (best < 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[k];
    }
  }
  r.count = nc;
  r.best = best;
  c->tile[f->order][f->precision] = best;
  if (rep) *rep = r;
  if (!c->tune_path.empty()) return write_tile_table(c);
  return ISR_OK;
}

int isr_submit(isr_ctx* c, const isr_field* f, uint64_t* req) {
  if (!c || !req) return fail(ISR_EINVAL, "ctx or req is NULL");
  int rc = check_field(f);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  return c->sched->submit(f, req);
}

int isr_poll(isr_ctx* c, uint64_t req, int32_t wait_ms, isr_blob** out, isr_stats* st) {
  if (!c) return fail(ISR_EINVAL, "ctx is NULL");
  if (out) *out = nullptr;
  return c->sched->poll(req, wait_ms, out, st);
}

int isr_decompress(isr_ctx* c, const isr_blob* b, void* d_out, int32_t out_prec, void* stream) {
  if (!c || !b || !d_out) return fail(ISR_EINVAL, "ctx, blob or output is NULL");
  if (out_prec != ISR_PREC_FP64 && out_prec != ISR_PREC_FP32) return fail(ISR_EINVAL, "out_prec must be FP64 or FP32");
  if (((uintptr_t)d_out) & 7) return fail(ISR_EINVAL, "output pointer is not 8-byte aligned");
  int rc = set_device(c);
  if (rc) return rc;
  Job j;
  std::memset(&j, 0, sizeof(j));
  j.n_elem = b->n_elem;
  j.order = b->order;
  j.ncomp = b->ncomp;
  j.vbytes = b->vbytes;
  j.tab = c->tab[b->order];
  j.bitmap = b->bitmap();
  j.elem_ptr = b->elem_ptr();
  j.values = b->values();
  j.voff = b->voff();
  if (b->value_kind == 1) j.qstep = b->qstep_dev();  // quantisation codes
  const int ofp64 = out_prec == ISR_PREC_FP64;
  hipStream_t s = (hipStream_t)stream;
  if (b->engine == ENG_GENERAL) {
    // FP64 blobs: the fixed-order FP64 inverse; FP32 / BF16 blobs of the
    // general passes: their MFMA inverse
    const long long total = (long long)tiles_per_comp(b->order, b->n_elem) * b->ncomp;
    const int grid = (int)std::min<long long>(total, (long long)c->num_cu * 8);
    HIPCHK(launch_pass(K_DECOMP, b->vbytes == 8 ? ISR_PREC_FP64 : b->precision, j, grid, s, d_out, ofp64));
    return ISR_OK;
  }
  // FP32 / BF16 blobs of the streaming engines: that engine's inverse, one
  // tile (or element) per wavefront
  j.tile = b->tile;
  const long long epw = b->engine == ENG_DENSE ? b->tile : fast_epw(b->order, 0);
  const long long waves = (b->n_elem + epw - 1) / epw * b->ncomp;
  const int grid = (int)std::max<long long>(1, std::min<long long>((waves + 3) / 4, (long long)c->num_cu * 8));
  const bool bf = b->precision == ISR_PREC_BF16;
  if (b->engine == ENG_DENSE)
    HIPCHK(bf ? launch_decomp_dense_bf16(j, grid, s, d_out, ofp64) : launch_decomp_dense_fp32(j, grid, s, d_out, ofp64));
  else
    HIPCHK(bf ? launch_decomp_wave_bf16(j, grid, s, d_out, ofp64) : launch_decomp_wave_fp32(j, grid, s, d_out, ofp64));
  return ISR_OK;
}

int isr_forward(isr_ctx* c, const isr_field* f, void* d_coef) {
  if (!c || !d_coef) return fail(ISR_EINVAL, "ctx or output is NULL");
  int rc = check_field(f);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->mu);
  Job j;
  std::memset(&j, 0, sizeof(j));
  const long long n = f->order + 1, n3 = n * n * n;
  j.u = f->field;
  j.comp_stride = f->comp_stride ? f->comp_stride : f->n_elem * n3;
  j.n_elem = f->n_elem;
  j.order = f->order;
  j.ncomp = f->ncomp;
  j.precision = f->precision;
  j.tab = c->tab[f->order];
  const long long total = (long long)tiles_per_comp(f->order, f->n_elem) * f->ncomp;
  const int grid = (int)std::min<long long>(total, (long long)c->num_cu * 8);
  hipStream_t s = (hipStream_t)f->stream;
  HIPCHK(launch_pass(K_FORWARD, f->precision, j, grid, s, d_coef));
  HIPCHK(hipStreamSynchronize(s));
  return ISR_OK;
}

int isr_blob_info(const isr_blob* b, int32_t* order, int32_t* ncomp, int64_t* n_elem, int32_t* value_bytes) {
  if (!b) return fail(ISR_EINVAL, "blob is NULL");
  if (order) *order = b->order;
  if (ncomp) *ncomp = b->ncomp;
  if (n_elem) *n_elem = b->n_elem;
  if (value_bytes) *value_bytes = b->vbytes;
  return ISR_OK;
}

int isr_blob_size(const isr_blob* b, uint64_t* bytes) {
  if (!b || !bytes) return fail(ISR_EINVAL, "blob or bytes is NULL");
  *bytes = b->serialized();
  return ISR_OK;
}

static void put_hdr(const isr_blob* b, char* p) {
  std::memcpy(p, "ISR1", 4);
  uint32_t ver = 3;
  std::memcpy(p + 4, &ver, 4);
  int32_t v32 = b->order;
  std::memcpy(p + 8, &v32, 4);
  v32 = b->ncomp;
  std::memcpy(p + 12, &v32, 4);
  int64_t ne = b->n_elem;
  std::memcpy(p + 16, &ne, 8);
  v32 = b->vbytes;
  std::memcpy(p + 24, &v32, 4);
  v32 = b->W;
  std::memcpy(p + 28, &v32, 4);
  std::memcpy(p + 32, &b->tol, 8);
  v32 = b->precision;
  std::memcpy(p + 40, &v32, 4);
  v32 = b->status;
  std::memcpy(p + 44, &v32, 4);
  v32 = b->engine;
  std::memcpy(p + 48, &v32, 4);
  v32 = b->tile;
  std::memcpy(p + 52, &v32, 4);
  v32 = b->value_kind;
  std::memcpy(p + 56, &v32, 4);
  v32 = 0;
  std::memcpy(p + 60, &v32, 4);
  for (int k = 0; k < b->ncomp; ++k) std::memcpy(p + isr_blob::HDR + isr_blob::CHDR * k, &b->comp[k], isr_blob::CHDR);
}

int isr_blob_to_host(const isr_blob* b, void* buf, uint64_t cap) {
  if (!b || !buf) return fail(ISR_EINVAL, "blob or buffer is NULL");
  const size_t need = b->serialized();
  if (cap < need) return fail(ISR_EINVAL, "buffer of %llu bytes is smaller than the blob (%zu)", (unsigned long long)cap, need);
  int rc = set_device(b->ctx);
  if (rc) return rc;
  char* p = (char*)buf;
  put_hdr(b, p);
  const size_t hb = isr_blob::HDR + isr_blob::CHDR * b->ncomp;
  const size_t body = b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
  HIPCHK(hipMemcpy(p + hb, b->bitmap(), body, hipMemcpyDeviceToHost));
  return ISR_OK;
}

int isr_blob_from_host(isr_ctx* c, const void* buf, uint64_t nbytes, isr_blob** out) {
  if (!c || !buf || !out) return fail(ISR_EINVAL, "ctx, buffer or out is NULL");
  *out = nullptr;
  const char* p = (const char*)buf;
  if (nbytes < isr_blob::HDR || std::memcmp(p, "ISR1", 4) != 0) return fail(ISR_EINVAL, "not an ISR1 blob");
  std::unique_ptr<isr_blob> b(new isr_blob());
  int32_t v32;
  int64_t ne;
  std::memcpy(&v32, p + 8, 4);
  b->order = v32;
  std::memcpy(&v32, p + 12, 4);
  b->ncomp = v32;
  std::memcpy(&ne, p + 16, 8);
  b->n_elem = ne;
  std::memcpy(&v32, p + 24, 4);
  b->vbytes = v32;
  std::memcpy(&v32, p + 28, 4);
  b->W = v32;
  std::memcpy(&b->tol, p + 32, 8);
  std::memcpy(&v32, p + 40, 4);
  b->precision = v32;
  std::memcpy(&v32, p + 44, 4);
  b->status = v32;
  uint32_t ver;
  std::memcpy(&ver, p + 4, 4);
  std::memcpy(&v32, p + 48, 4);
  b->engine = v32;
  std::memcpy(&v32, p + 52, 4);
  b->tile = v32;
  std::memcpy(&v32, p + 56, 4);
  b->value_kind = v32;
  if (ver != 3) return fail(ISR_EINVAL, "blob version %u is not 3", ver);
  if (b->value_kind != 0 && !(b->value_kind == 1 && b->vbytes == 4 && b->precision == ISR_PREC_FP64))
    return fail(ISR_EINVAL, "corrupt blob header (value kind %d)", b->value_kind);
  if (b->order < 1 || b->order > ISR_MAX_ORDER || b->ncomp < 1 || b->ncomp > ISR_MAX_COMP || b->n_elem < 1 ||
      (b->vbytes != 4 && b->vbytes != 8) || b->W != words_per_elem(b->order) ||
      (b->vbytes == 8) != (b->precision == ISR_PREC_FP64 && b->value_kind == 0) ||
      (b->precision != ISR_PREC_FP64 && b->precision != ISR_PREC_FP32 && b->precision != ISR_PREC_BF16))
    return fail(ISR_EINVAL, "corrupt blob header");
  if ((b->engine == ENG_GENERAL && b->tile != 0) ||
      (b->engine == ENG_WAVE && (b->tile != 0 || !fast_order(b->order, b->precision) || b->precision == ISR_PREC_FP64)) ||
      (b->engine == ENG_DENSE && (!dense_shape(b->order, b->tile) || b->precision == ISR_PREC_FP64)) ||
      b->engine < ENG_GENERAL || b->engine > ENG_DENSE)
    return fail(ISR_EINVAL, "corrupt blob header (engine %d, tile %d)", b->engine, b->tile);
  if (nbytes < isr_blob::HDR + isr_blob::CHDR * (size_t)b->ncomp) return fail(ISR_EINVAL, "truncated blob");
  uint64_t tk = 0;
  for (int k = 0; k < b->ncomp; ++k) {
    std::memcpy(&b->comp[k], p + isr_blob::HDR + isr_blob::CHDR * k, isr_blob::CHDR);
    if (b->comp[k].voff != tk) return fail(ISR_EINVAL, "corrupt blob component offsets");
    tk += b->comp[k].kept;
  }
  b->total_kept = tk;
  if (nbytes != b->serialized()) return fail(ISR_EINVAL, "blob size %llu does not match its header (%zu)", (unsigned long long)nbytes, b->serialized());
  // the offset tables must agree with the bitmaps and the kept counts, since
  // decompression indexes the values with them
  {
    const size_t hb0 = isr_blob::HDR + isr_blob::CHDR * b->ncomp;
    const u64* bm = (const u64*)(p + hb0);
    const u64* ep = (const u64*)(p + hb0 + b->bitmap_bytes());
    for (int k = 0; k < b->ncomp; ++k) {
      const u64* e = ep + (size_t)k * (b->n_elem + 1);
      const u64* m = bm + (size_t)k * b->n_elem * b->W;
      if (e[0] != 0 || e[b->n_elem] != b->comp[k].kept) return fail(ISR_EINVAL, "corrupt blob offset table");
      for (int64_t q = 0; q < b->n_elem; ++q) {
        u64 pc = 0;
        for (int w = 0; w < b->W; ++w) pc += (u64)__builtin_popcountll(m[q * b->W + w]);
        if (e[q + 1] < e[q] || e[q + 1] - e[q] != pc) return fail(ISR_EINVAL, "corrupt blob bitmap or offsets");
      }
    }
  }
  int rc = set_device(c);
  if (rc) return rc;
  b->ctx = c;
  b->dev_bytes = 256 + b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
  b->dev = c->arena->alloc(b->dev_bytes, true);
  if (!b->dev) return fail(ISR_ENOMEM, "blob does not fit the HBM budget");
  u64 vo[ISR_MAX_COMP];
  for (int k = 0; k < b->ncomp; ++k) vo[k] = b->comp[k].voff;
  const size_t hb = isr_blob::HDR + isr_blob::CHDR * b->ncomp;
  double qs[ISR_MAX_COMP];
  for (int k = 0; k < b->ncomp; ++k) qs[k] = b->comp[k].qstep;
  if (hipMemcpy(b->qstep_dev(), qs, 8 * b->ncomp, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->voff(), vo, 8 * b->ncomp, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->bitmap(), p + hb, nbytes - hb, hipMemcpyHostToDevice) != hipSuccess) {
    c->arena->free(b->dev);
    return fail(ISR_EDEVICE, "blob upload failed");
  }
  *out = b.release();
  return ISR_OK;
}

int isr_pack_submit(isr_ctx* c, const isr_blob* b, int32_t codec, int32_t level, uint32_t flags, uint64_t* job) {
  if (!c || !b || !job) return fail(ISR_EINVAL, "ctx, blob or job is NULL");
  if (b->ctx != c) return fail(ISR_EINVAL, "the blob belongs to another context");
  if ((codec != ISR_CODEC_ZLIB || level < 0 || level > 9) && (codec != ISR_CODEC_BZIP2 || level < 1 || level > 9))
    return fail(ISR_EINVAL, "codec %d with level %d is not supported (zlib 0-9, bzip2 1-9)", codec, level);
  if (flags & ~(uint32_t)ISR_PACK_SHUFFLE) return fail(ISR_EINVAL, "unknown packing flags 0x%x", flags);
  int rc = set_device(c);
  if (rc) return rc;
  char hdr[isr_blob::HDR + isr_blob::CHDR * ISR_MAX_COMP];
  put_hdr(b, hdr);
  const size_t hb = isr_blob::HDR + isr_blob::CHDR * b->ncomp;
  const size_t body = b->bitmap_bytes() + b->ptr_bytes() + b->values_bytes();
  try {
    return isr::packer_submit(c->packer, (const unsigned char*)hdr, hb, b->bitmap(), body, codec, level, flags, job);
  } catch (...) {  // no C++ exception crosses the C ABI
    return fail(ISR_ENOMEM, "could not queue the blob for the lossless stage");
  }
}

int isr_pack_poll(isr_ctx* c, uint64_t job, int32_t wait_ms, void* out, uint64_t cap, uint64_t* out_bytes,
                  double* seconds) {
  if (!c) return fail(ISR_EINVAL, "ctx is NULL");
  try {
    return isr::packer_poll(c->packer, job, wait_ms, out, cap, out_bytes, seconds);
  } catch (...) {
    return fail(ISR_ENOMEM, "could not collect the packed blob");
  }
}

void isr_blob_free(isr_blob* b) {
  if (!b) return;
  if (b->ctx && b->dev) {
    (void)hipSetDevice(b->ctx->device);
    b->ctx->arena->free(b->dev);
  }
  delete b;
}

int isr_gll_tables(int32_t order, double* xi, double* w, double* V, double* A, double* gamma, double* w3,
                   double* g3) {
  HostTables t;
  if (!host_tables(order, &t)) return fail(ISR_EINVAL, "order %d outside [1, %d]", order, ISR_MAX_ORDER);
  const int n = order + 1, n2 = n * n, n3 = n2 * n;
  if (xi) std::memcpy(xi, t.xi, n * 8);
  if (w) std::memcpy(w, t.w, n * 8);
  if (gamma) std::memcpy(gamma, t.gamma, n * 8);
  if (V) std::memcpy(V, t.V, n2 * 8);
  if (A) std::memcpy(A, t.A, n2 * 8);
  if (w3) std::memcpy(w3, t.w3, n3 * 8);
  if (g3) std::memcpy(g3, t.g3, n3 * 8);
  return ISR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free compression (isr_compress_noalloc)

namespace isr {

int run_compress_noalloc(isr_ctx* c, const isr_field* f, char* scratch, size_t scratch_cap, void* d_out,
                         uint64_t out_cap, uint64_t* out_bytes, isr_stats* st) {
  const double t0 = now_s();
  int rc = check_field(f);
  if (rc) return rc;
  if (!d_out) return fail(ISR_EINVAL, "output pointer is NULL");
  if (((uintptr_t)d_out) & 255) return fail(ISR_EINVAL, "output pointer is not 256-byte aligned");
  std::lock_guard<std::mutex> g(c->mu);
  const Sizes z = plan_sizes(f, ctx_tile(c, f->order, f->precision));
  const int nc = f->ncomp;
  const size_t hb = isr_blob::HDR + isr_blob::CHDR * (size_t)nc;
  const size_t bm = (size_t)nc * f->n_elem * z.W * 8, ep = (size_t)nc * (f->n_elem + 1) * 8;
  const size_t need = hb + bm + ep + (size_t)nc * z.nv * z.vbytes;
  if (out_bytes) *out_bytes = need;
  if (out_cap < need)
    return fail(ISR_EINVAL, "output buffer of %llu bytes is smaller than the worst-case blob of %zu bytes",
                (unsigned long long)out_cap, need);
  // the per-component value offsets live right after the scratch proper
  const size_t voff_at = (z.scratch_bytes + 255) & ~size_t(255);
  if (voff_at + 256 > scratch_cap)
    return fail(ISR_ENOMEM, "request needs %zu bytes of scratch; the allocation-free entry point holds %zu",
                voff_at + 256, scratch_cap);
  char* out = (char*)d_out;
  const BlobPtrs bp{(u64*)(scratch + voff_at), (u64*)(out + hb), (u64*)(out + hb + bm), out + hb + bm + ep};
  Job j = make_job(c, f, z, scratch, bp);
  hipStream_t s = (hipStream_t)f->stream;
  CompState* hs = c->st_host;
  bool fast = z.fast;
  int iters = 0;
  for (;;) {
    rc = enqueue_pipeline(c, j, z, s, nullptr, fast);
    if (rc) return rc;
    HIPCHK(launch_state_out(j.st, hs, nc, s));
    HIPCHK(hipStreamSynchronize(s));
    int flags = 0;
    for (int k = 0; k < nc; ++k) flags |= hs[k].flags;
    if (fast && (flags & ST_MISS)) {  // threshold outside the sampled window: general pipeline
      fast = false;
      j.sample_stride = 0;
      continue;
    }
    rc = status_from_flags(flags);
    if (rc) return rc;
    if (!plan_repair(f, hs, iters, j.Bov)) break;
    ++iters;
  }
  // describe the result in a blob record on the stack (no device memory of
  // its own) to form the header
  isr_blob b;
  std::memset(b.comp, 0, sizeof(b.comp));  // records not set below (the quantisation step) stay 0
  b.ctx = c;
  b.order = f->order;
  b.ncomp = nc;
  b.n_elem = f->n_elem;
  b.vbytes = z.vbytes;
  b.W = z.W;
  b.tol = f->tol;
  b.precision = f->precision;
  isr_stats tmp;
  std::memset(&tmp, 0, sizeof(tmp));
  fill_stats(&b, hs, &tmp);
  bool within = true;
  if (f->tol >= 0.0)
    for (int k = 0; k < nc; ++k) within = within && !(hs[k].rel > f->tol);
  b.status = within ? ISR_OK : ISR_ETOL;
  set_engine(&b, fast, z.tile);
  char hdr[isr_blob::HDR + isr_blob::CHDR * ISR_MAX_COMP];
  put_hdr(&b, hdr);
  HIPCHK(launch_put_bytes(hdr, (int)hb, d_out, s));
  HIPCHK(hipStreamSynchronize(s));
  if (out_bytes) *out_bytes = b.serialized();
  tmp.repair_iters = iters;
  tmp.path = fast ? 1 : 0;
  tmp.status = b.status;
  tmp.t_submit = t0;
  tmp.t_start = t0;
  tmp.t_done = now_s();
  if (st) *st = tmp;
  if (!within) fail(ISR_ETOL, "relative error above tol after %d repairs", iters);
  return b.status;
}

}  // namespace isr

// ---------------------------------------------------------------------------
// quantised variant (isr_compress_quantized)

namespace isr {

// The cut of the plain FP64 method at ((tol*tol)*U2)*(1 - share), then the
// kept coefficients quantised with the step 2 sqrt((B - S_c)/K)(1 - 2^-20)
// that the rest of the budget B = (tol*tol)*U2 allows, the exact error of the
// dequantised field measured, and the step shrunk by (tol/rel)(1 - 2^-20)
// while rounding leaves it above tol (at most 4 times).
int run_compress_quantized(isr_ctx* c, const isr_field* f, double share, isr_blob** out, isr_stats* st) {
  *out = nullptr;
  int rc = check_field(f);
  if (rc) return rc;
  if (f->precision != ISR_PREC_FP64) return fail(ISR_EINVAL, "the quantised variant runs on the FP64 path");
  if (f->elem_jac) return fail(ISR_EINVAL, "the quantised variant takes unit Jacobians (elem_jac NULL)");
  if (!(f->tol >= 0.0)) return fail(ISR_EINVAL, "the quantised variant needs tol >= 0");
  if (!(share >= 0.0 && share < 1.0)) return fail(ISR_EINVAL, "share must be in [0, 1)");
  const double t0 = now_s();
  isr_blob* b = nullptr;
  isr_stats s0;
  rc = run_compress(c, f, &b, &s0, 1.0 - share);
  if (rc != ISR_OK) {
    if (b) isr_blob_free(b);
    return rc;
  }
  const int nc = f->ncomp;
  hipStream_t s = (hipStream_t)f->stream;
  double delta[ISR_MAX_COMP], Bf[ISR_MAX_COMP], err2[ISR_MAX_COMP], rel[ISR_MAX_COMP];
  for (int k = 0; k < nc; ++k) {
    Bf[k] = (f->tol * f->tol) * b->comp[k].U2;
    const uint64_t K = b->comp[k].kept;
    delta[k] = K ? (2.0 * std::sqrt((Bf[k] - b->comp[k].dropped) / (double)K)) * (1.0 - 0x1p-20) : 0.0;
  }
  // the quantised blob: the cut's bitmaps and offsets, FP32 codes
  isr_blob* q = new isr_blob();
  *q = *b;
  q->vbytes = 4;
  q->value_kind = 1;
  q->engine = ENG_GENERAL;
  q->tile = 0;
  q->dev_bytes = 256 + q->bitmap_bytes() + q->ptr_bytes() + q->values_bytes();
  q->dev = c->arena->alloc(q->dev_bytes, true);
  const size_t hist_bytes = (size_t)nc * HBINS * sizeof(HistBin);
  char* scr = (char*)c->arena->alloc(hist_bytes + 512);
  auto cleanup = [&]() {
    if (scr) c->arena->free(scr);
    isr_blob_free(b);
  };
  if (!q->dev || !scr) {
    if (q->dev) c->arena->free(q->dev);
    delete q;
    cleanup();
    return fail(ISR_ENOMEM, "the quantised blob does not fit the HBM budget");
  }
  Job j;
  std::memset(&j, 0, sizeof(j));
  const long long n = f->order + 1, n3 = n * n * n;
  j.u = f->field;
  j.comp_stride = f->comp_stride ? f->comp_stride : f->n_elem * n3;
  j.n_elem = f->n_elem;
  j.order = f->order;
  j.ncomp = nc;
  j.precision = ISR_PREC_FP64;
  j.vbytes = 8;
  j.tab = c->tab[f->order];
  j.bitmap = b->bitmap();
  j.elem_ptr = b->elem_ptr();
  j.values = b->values();
  j.voff = b->voff();
  j.qstep = q->qstep_dev();
  j.qvals = (float*)q->values();
  j.histR = (HistBin*)scr;
  j.ticket = (u32*)(scr + hist_bytes);
  double* err_dev = (double*)(scr + hist_bytes + 256);
  const long long total = (long long)tiles_per_comp(f->order, f->n_elem) * nc;
  const int grid = (int)std::min<long long>(total, (long long)c->num_cu * resident_blocks(K_PASS3, ISR_PREC_FP64, f->order));
  int iters = 0;
  for (;;) {
    uint32_t over = 0;
    rc = ISR_OK;
    if (launch_zero(scr, hist_bytes + 256, s) != hipSuccess ||
        hipMemcpyAsync((void*)j.qstep, delta, 8 * nc, hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_pass(K_QUANT, ISR_PREC_FP64, j, grid, s) != hipSuccess || launch_err_total(j, err_dev, s) != hipSuccess ||
        hipMemcpyAsync(err2, err_dev, 8 * nc, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&over, j.ticket + 1, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = fail(ISR_EDEVICE, "quantisation pass failed: %s", hipGetErrorString(hipGetLastError()));
    if (!rc && over) rc = fail(ISR_ETOL, "a quantisation code needs more than 24 bits at this step");
    if (rc) {
      c->arena->free(q->dev);
      delete q;
      cleanup();
      return rc;
    }
    bool again = false;
    for (int k = 0; k < nc; ++k) {
      rel[k] = q->comp[k].U2 > 0.0 ? std::sqrt(err2[k] / q->comp[k].U2) : 0.0;
      if (rel[k] > f->tol && iters < 4) {
        delta[k] = (delta[k] * (f->tol / rel[k])) * (1.0 - 0x1p-20);
        again = true;
      }
    }
    if (!again) break;
    ++iters;
  }
  // the blob's bitmaps, offsets and value offsets are the cut's
  if (hipMemcpyAsync(q->voff(), b->voff(), 64, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(q->bitmap(), b->bitmap(), q->bitmap_bytes() + q->ptr_bytes(), hipMemcpyDeviceToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    c->arena->free(q->dev);
    delete q;
    cleanup();
    return fail(ISR_EDEVICE, "quantised blob copy failed");
  }
  bool within = true;
  for (int k = 0; k < nc; ++k) {
    q->comp[k].B = Bf[k];
    q->comp[k].err2 = err2[k];
    q->comp[k].rel = rel[k];
    q->comp[k].qstep = delta[k];
    within = within && !(rel[k] > f->tol);
  }
  q->status = within ? ISR_OK : ISR_ETOL;
  cleanup();
  if (st) {
    *st = s0;
    for (int k = 0; k < nc; ++k) {
      st->budget[k] = Bf[k];
      st->err2[k] = err2[k];
      st->rel_err[k] = rel[k];
    }
    st->blob_bytes = q->serialized();
    st->cr = st->in_bytes ? (double)((int64_t)st->in_bytes - (int64_t)st->blob_bytes) / (double)st->in_bytes : 0.0;
    st->repair_iters = iters;
    st->status = q->status;
    st->t_submit = t0;
    st->t_done = now_s();
  }
  *out = q;
  if (!within) fail(ISR_ETOL, "relative error above tol after %d step repairs", iters);
  return q->status;
}


// Per-element cut: every element cut alone at ((tol*tol)*U2_e)*s_c; pass 3
// of the general pipeline compacts, inverts and measures the exact error;
// s_c follows the plain budget repair while rounding leaves rel above tol.
int run_compress_elemcut(isr_ctx* c, const isr_field* f, isr_blob** out, isr_stats* st) {
  *out = nullptr;
  int rc = check_field(f);
  if (rc) return rc;
  if (f->precision != ISR_PREC_FP64) return fail(ISR_EINVAL, "the per-element cut runs on the FP64 path");
  if (!(f->tol >= 0.0)) return fail(ISR_EINVAL, "the per-element cut needs tol >= 0");
  if (f->n_elem >= (1ll << 32)) return fail(ISR_EINVAL, "the per-element cut takes fewer than 2^32 elements");
  const double t0 = now_s();
  const int nc = f->ncomp;
  const long long n = f->order + 1, n3 = n * n * n, E = f->n_elem;
  const int W = (int)((n3 + 63) / 64);
  hipStream_t s = (hipStream_t)f->stream;
  isr_blob* b = new isr_blob();
  b->ctx = c;
  b->order = f->order;
  b->ncomp = nc;
  b->n_elem = E;
  b->vbytes = 8;
  b->W = W;
  b->tol = f->tol;
  b->precision = ISR_PREC_FP64;
  b->engine = ENG_GENERAL;
  b->dev_bytes = 256 + (size_t)nc * E * W * 8 + (size_t)nc * (E + 1) * 8 + (size_t)nc * E * n3 * 8;
  b->dev = c->arena->alloc(b->dev_bytes, true);
  const long long tiles = tiles_per_comp(f->order, E);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_coef = 0, o_tau = al(o_coef + (size_t)nc * E * n3 * 8), o_st = al(o_tau + (size_t)nc * E * 8);
  const size_t o_zero = al(o_st + (size_t)nc * sizeof(CompState));  // digits, error bins, look-back, ticket
  const size_t o_hist = al(o_zero + elemcut_digit_bytes(nc));
  const size_t o_lb = al(o_hist + (size_t)nc * HBINS * sizeof(HistBin));
  const size_t o_tk = al(o_lb + (size_t)nc * tiles * 8);
  const size_t scr_bytes = o_tk + 256;
  char* scr = b->dev ? (char*)c->arena->alloc(scr_bytes) : nullptr;
  if (!b->dev || !scr) {
    if (b->dev) c->arena->free(b->dev);
    delete b;
    return fail(ISR_ENOMEM, "the per-element cut does not fit the HBM budget");
  }
  auto give_up = [&](int code) {
    c->arena->free(scr);
    isr_blob_free(b);
    return code;
  };
  Job j;
  std::memset(&j, 0, sizeof(j));
  j.u = f->field;
  j.jac = f->elem_jac;
  j.comp_stride = f->comp_stride ? f->comp_stride : E * n3;
  j.n_elem = E;
  j.order = f->order;
  j.ncomp = nc;
  j.precision = ISR_PREC_FP64;
  j.vbytes = 8;
  j.tol = f->tol;
  j.cut_scale = 1.0;
  for (int k = 0; k < 8; ++k) j.Bov[k] = -1.0;
  j.tab = c->tab[f->order];
  j.st = (CompState*)(scr + o_st);
  j.histR = (HistBin*)(scr + o_hist);
  j.lookback = (u64*)(scr + o_lb);
  j.ticket = (u32*)(scr + o_tk);
  j.bitmap = b->bitmap();
  j.elem_ptr = b->elem_ptr();
  j.values = b->values();
  j.voff = b->voff();
  j.tau_elem = (const double*)(scr + o_tau);
  double* coef = (double*)(scr + o_coef);
  const int gfwd = (int)std::min<long long>(tiles * nc, (long long)c->num_cu * 8);
  if (launch_pass(K_FORWARD, ISR_PREC_FP64, j, gfwd, s, coef) != hipSuccess)
    return give_up(fail(ISR_EDEVICE, "forward transform failed: %s", hipGetErrorString(hipGetLastError())));
  const int gsel = (int)std::max<long long>(1, std::min<long long>((E * nc + 3) / 4, (long long)c->num_cu * 8));
  const int g3 = (int)std::min<long long>(tiles * nc, (long long)c->num_cu * resident_blocks(K_PASS3, ISR_PREC_FP64, f->order));
  double scale[ISR_MAX_COMP];
  for (int k = 0; k < ISR_MAX_COMP; ++k) scale[k] = 1.0;
  CompState hs[ISR_MAX_COMP];
  int iters = 0;
  for (;;) {
    std::memset(hs, 0, sizeof(hs));
    for (int k = 0; k < nc; ++k) {
      hs[k].tol = f->tol;
      hs[k].n_values = (u64)(E * n3);
      hs[k].bstar = -1;
    }
    if (hipMemcpyAsync(j.st, hs, nc * sizeof(CompState), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_zero(scr + o_zero, o_tk + 256 - o_zero, s) != hipSuccess ||
        launch_elemcut(j, coef, (double*)(scr + o_tau), (u64*)(scr + o_zero), scale, gsel, s) != hipSuccess ||
        launch_pass(K_PASS3, ISR_PREC_FP64, j, g3, s) != hipSuccess || launch_finalize(j, s) != hipSuccess ||
        hipMemcpyAsync(hs, j.st, nc * sizeof(CompState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return give_up(fail(ISR_EDEVICE, "per-element cut failed: %s", hipGetErrorString(hipGetLastError())));
    int flags = 0;
    for (int k = 0; k < nc; ++k) flags |= hs[k].flags;
    rc = status_from_flags(flags);
    if (rc) return give_up(rc);
    bool again = false;
    if (iters < 4) {
      for (int k = 0; k < nc; ++k) {
        if (hs[k].rel > f->tol) {
          const double fr = f->tol / hs[k].rel;
          scale[k] = (scale[k] * (fr * fr)) * (1.0 - 0x1p-20);
          again = true;
        }
      }
    }
    if (!again) break;
    ++iters;
  }
  fill_stats(b, hs, st);
  bool within = true;
  for (int k = 0; k < nc; ++k) within = within && !(hs[k].rel > f->tol);
  b->status = within ? ISR_OK : ISR_ETOL;
  c->arena->free(scr);
  if (st) {
    st->repair_iters = iters;
    st->status = b->status;
    st->t_submit = t0;
    st->t_done = now_s();
  }
  *out = b;
  if (!within) fail(ISR_ETOL, "relative error above tol after %d budget repairs", iters);
  return b->status;
}

}  // namespace isr

extern "C" int isr_compress_quantized(isr_ctx* c, const isr_field* f, double share, isr_blob** out, isr_stats* st) {
  if (!c || !out) return fail(ISR_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  if (st) std::memset(st, 0, sizeof(*st));
  int rc = set_device(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->mu);
  return isr::run_compress_quantized(c, f, share, out, st);
}

extern "C" int isr_compress_elemcut(isr_ctx* c, const isr_field* f, isr_blob** out, isr_stats* st) {
  if (!c || !out) return fail(ISR_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  if (st) std::memset(st, 0, sizeof(*st));
  int rc = set_device(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->mu);
  return isr::run_compress_elemcut(c, f, out, st);
}
