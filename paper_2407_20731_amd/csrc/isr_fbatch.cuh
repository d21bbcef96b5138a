// One persistent launch over a batch of FP32 / BF16 snapshots (orders 5, 7, 9,
// uneven sizes, each with the tile shape its context holds for it: built-in
// or autotuned) on the streaming path.
//
// The queue is phase-major, like the FP64 batch kernel's (isr_batch.cuh):
//   sample, pass A, gather + level-1 select, refinement levels 2..6, counts,
//   offset scans (two), pass B + finalize
// and each phase holds the items of every (snapshot, component) pair.  An item
// is one workgroup of the phase's per-launch grid: it runs the same device body
// with the same virtual workgroup index and count as the per-phase launch, so
// every snapshot's results are bit-identical to compressing it alone.  An item
// waits (bounded spin) only on counters of earlier phases: its own pair's
// previous phase, and for pass B also the last selection of every component
// of its snapshot (the value offsets of the earlier components).  Items of
// earlier phases hold smaller tickets, so they were claimed by workgroups that
// are already running and never wait on later tickets.
#pragma once

#include "isr_batch.cuh"
#include "isr_engine_d.cuh"
#include "isr_fastsel.cuh"

namespace isr {

// The batch kernel's dynamic LDS; every body function names it itself, so
// that its accesses stay LDS instructions (a pointer passed as an argument
// would be a generic one).
extern __shared__ __align__(16) unsigned char fb_lds[];

// A body function gets its job from the batch table through a wave-uniform
// address and works on a private copy: the fields land in scalar registers
// and, as with a kernel argument, no store of the body can change them.
// Its pointers go through the global address space, which lets the compiler
// use global instead of generic memory instructions, as it does for the
// pointers of a kernel argument.
template <class T>
DEV T* fb_global(T* p) {
  typedef __attribute__((address_space(1))) T GT;
  return (T*)(GT*)p;
}
DEV Job fb_job(const Job* jr) {
  const u64 a = (u64)(uintptr_t)jr;
  const u32 lo = (u32)__builtin_amdgcn_readfirstlane((int)(u32)a);
  const u32 hi = (u32)__builtin_amdgcn_readfirstlane((int)(u32)(a >> 32));
  Job j = *(const Job*)(uintptr_t)(((u64)hi << 32) | lo);
  j.u = fb_global(j.u);
  j.jac = fb_global(j.jac);
  j.tab.A = fb_global(j.tab.A);
  j.tab.V = fb_global(j.tab.V);
  j.tab.w3 = fb_global(j.tab.w3);
  j.tab.g3 = fb_global(j.tab.g3);
  j.tab.A32 = fb_global(j.tab.A32);
  j.tab.V32 = fb_global(j.tab.V32);
  j.histE = fb_global(j.histE);
  j.histN = fb_global(j.histN);
  j.histR = fb_global(j.histR);
  j.histL = fb_global(j.histL);
  j.histEs = fb_global(j.histEs);
  j.histNs = fb_global(j.histNs);
  j.st = fb_global(j.st);
  j.lists = fb_global(j.lists);
  j.lidx = fb_global(j.lidx);
  j.cnt = fb_global(j.cnt);
  j.slotsA = fb_global(j.slotsA);
  j.slotsB = fb_global(j.slotsB);
  j.done = fb_global(j.done);
  j.chunk = fb_global(j.chunk);
  j.lookback = fb_global(j.lookback);
  j.ticket = fb_global(j.ticket);
  j.bitmap = fb_global(j.bitmap);
  j.elem_ptr = fb_global(j.elem_ptr);
  j.values = fb_global(j.values);
  j.voff = fb_global(j.voff);
  return j;
}
DEV int fb_u(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Bodies of one (order, tile shape) in the persistent kernel: the dense-tile
// engine (T > 0), the wave-tile engine (T = 0, orders up to 7) or the
// large-order engine (T = 0, orders 8..11).  Every shape the autotuner may
// pick for orders 5, 7 and 9 is here (ISR_FBATCH_SHAPES).
template <int N, int PREC, int T>
struct FbOrder {
  typedef SampleLdsD<N, PREC, T> LS;
  typedef PassALdsD<N, PREC, T> LA;
  typedef PassBLdsD<N, PREC, T> LB;
  static DEV void sample(const Job& j, int c, int k, int nk) { sampleD_body<N, PREC, T>(j, c, k, nk, *(LS*)fb_lds, true); }
  static DEV void passA(const Job& j, int c, int k, int nk) { passAD_body<N, PREC, T>(j, c, k, nk, *(LA*)fb_lds); }
  static DEV void passB(const Job& j, int c, int k, int nk) { passBD_body<N, PREC, T>(j, c, k, nk, *(LB*)fb_lds, true); }
};
template <int N, int PREC>
struct FbWave {
  typedef SampleLds<N, PREC> LS;
  typedef PassALds<N, PREC> LA;
  typedef PassBLds<N, PREC> LB;
  static DEV void sample(const Job& j, int c, int k, int nk) { sample_body<N, PREC>(j, c, k, nk, *(LS*)fb_lds, true); }
  static DEV void passA(const Job& j, int c, int k, int nk) { passA_body<N, PREC>(j, c, k, nk, *(LA*)fb_lds); }
  static DEV void passB(const Job& j, int c, int k, int nk) { passB_body<N, PREC>(j, c, k, nk, *(LB*)fb_lds, true); }
};
template <int N, int PREC>
struct FbLarge {
  typedef SampleLdsL<N, PREC> LS;
  typedef PassALdsL<N, PREC> LA;
  typedef PassBLdsL<N, PREC> LB;
  static DEV void sample(const Job& j, int c, int k, int nk) { sampleL_body<N, PREC>(j, c, k, nk, *(LS*)fb_lds, true); }
  static DEV void passA(const Job& j, int c, int k, int nk) { passAL_body<N, PREC>(j, c, k, nk, *(LA*)fb_lds); }
  static DEV void passB(const Job& j, int c, int k, int nk) { passBL_body<N, PREC>(j, c, k, nk, *(LB*)fb_lds, true); }
};
template <int N, int PREC, int T>
struct FbSel {
  typedef FbOrder<N, PREC, T> type;
};
template <int N, int PREC>
struct FbSel<N, PREC, 0> {
  typedef typename Pick<(N <= FAST_MAX_ORDER), FbWave<N, PREC>, FbLarge<N, PREC>>::type type;
};

// Each body is its own (not inlined) function: the registers of one phase do
// not constrain another's, and the kernel needs the largest of them only.
template <class F>
__device__ __noinline__ void fb_sample(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  F::sample(j, fb_u(comp), fb_u(k), fb_u(nk));
}
template <class F>
__device__ __noinline__ void fb_passA(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  F::passA(j, fb_u(comp), fb_u(k), fb_u(nk));
}
template <class F>
__device__ __noinline__ void fb_passB(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  F::passB(j, fb_u(comp), fb_u(k), fb_u(nk));
}
__device__ __noinline__ void fb_gather(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  gather_body(j, fb_u(comp), fb_u(k), fb_u(nk), *reinterpret_cast<GatherLds*>(fb_lds), true);
}
__device__ __noinline__ void fb_refsel(const Job* jr, int comp, int L, int k, int nk) {
  const Job j = fb_job(jr);
  refsel_body(j, fb_u(comp), fb_u(L), fb_u(k), fb_u(nk), *reinterpret_cast<RefselLds*>(fb_lds));
}
__device__ __noinline__ void fb_count(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  count_body(j, fb_u(comp), fb_u(k), fb_u(nk));
}
__device__ __noinline__ void fb_scan1(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  scan1_body(j, fb_u(comp), fb_u(k), fb_u(nk), *reinterpret_cast<ScanLds*>(fb_lds));
}
__device__ __noinline__ void fb_scan2(const Job* jr, int comp, int k, int nk) {
  const Job j = fb_job(jr);
  scan2_body(j, fb_u(comp), fb_u(k), fb_u(nk), *reinterpret_cast<ScanLds*>(fb_lds));
}

template <class F>
DEV void fb_engine(int ph, const Job* j, int comp, int k, int nk) {
  if (ph == FQ_SAMPLE)
    fb_sample<F>(j, comp, k, nk);
  else if (ph == FQ_PASSA)
    fb_passA<F>(j, comp, k, nk);
  else
    fb_passB<F>(j, comp, k, nk);
}

template <int PREC>
__global__ __launch_bounds__(256, 3) void k_fbatch(BatchCtl B) {
  __shared__ long long tk_s;
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  const long long total = B.phase_off[NFQ];
  for (;;) {
    __syncthreads();
    if (tid == 0) tk_s = (long long)atomicAdd(B.ticket, 1ull);
    __syncthreads();
    const long long tk = tk_s;
    if (tk >= total) break;
    int ph = 0;
    while (tk >= B.phase_off[ph + 1]) ++ph;
    const long long x = tk - B.phase_off[ph];
    const long long* row = B.items + (size_t)ph * (B.npairs + 1);
    int lo = 0, hi = B.npairs;  // row[lo] <= x < row[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (row[mid] <= x)
        lo = mid;
      else
        hi = mid;
    }
    const int q = lo;
    const int k = (int)(x - row[q]);
    const int nk = (int)(row[q + 1] - row[q]);
    const int snap = B.pair_snap[q], comp = B.pair_comp[q];
    const Job* jp = B.jobs + snap;
    const Job& j = *jp;
    if (tid == 0) {
      bool ok = true;
      if (ph == FQ_PASSB) {
        ok = wait_count(&B.done[(size_t)FQ_SCAN2 * B.npairs + q], (u32)items_of(B, FQ_SCAN2, q));
        const int q0 = q - comp;
        for (int cc = 0; cc < j.ncomp && ok; ++cc)
          ok = wait_count(&B.done[(size_t)FQ_R6 * B.npairs + q0 + cc], (u32)items_of(B, FQ_R6, q0 + cc));
      } else if (ph > 0) {
        ok = wait_count(&B.done[(size_t)(ph - 1) * B.npairs + q], (u32)items_of(B, ph - 1, q));
      }
      ok_s = ok;
      if (!ok) atomicOr(B.err, 1);
    }
    __syncthreads();
    if (ok_s) {
      if (ph == FQ_SAMPLE || ph == FQ_PASSA || ph == FQ_PASSB) {
        const int o = j.order, t = j.tile;
#define FB_CASE(O, T)                                                 \
  if (o == O && t == T) {                                             \
    fb_engine<typename FbSel<O, PREC, T>::type>(ph, jp, comp, k, nk); \
  } else
        ISR_FBATCH_SHAPES(FB_CASE) {
          if (tid == 0) atomicOr(B.err, 2);  // a shape the host never enqueues
        }
#undef FB_CASE
      } else if (ph == FQ_GATHER) {
        fb_gather(jp, comp, k, nk);
      } else if (ph == FQ_COUNT) {
        fb_count(jp, comp, k, nk);
      } else if (ph == FQ_SCAN1) {
        fb_scan1(jp, comp, k, nk);
      } else if (ph == FQ_SCAN2) {
        fb_scan2(jp, comp, k, nk);
      } else {
        fb_refsel(jp, comp, 2 + (ph - FQ_R2), k, nk);
      }
    }
    // a dependency that never completed (cannot happen) skips the work and
    // keeps the queue draining; the host reports it
    __syncthreads();
    if (tid == 0) add_rel32(&B.done[(size_t)ph * B.npairs + q], 1u);
  }
}

template <int PREC>
hipError_t launch_fbatch_prec(const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_fbatch<PREC>, dim3(grid), dim3(256), lds_bytes, s, B);
  return hipGetLastError();
}

template <class T>
constexpr size_t fb_max(size_t m) {
  return m > sizeof(T) ? m : sizeof(T);
}

// Dynamic LDS of the persistent kernel: order 0 gives the order-independent
// phases' share, (order, tile) that shape's bodies'; a batch launches with the
// largest over the shapes it holds.
template <int PREC>
size_t fbatch_lds_prec(int order, int tile) {
  size_t m = 0;
  if (order == 0) {
    m = sizeof(GatherLds);
    m = fb_max<RefselLds>(m);
    m = fb_max<ScanLds>(m);
  }
#define FB_LDS(O, T)                                   \
  if (order == O && tile == T) {                       \
    typedef typename FbSel<O, PREC, T>::type F;        \
    m = fb_max<typename F::LS>(m);                     \
    m = fb_max<typename F::LA>(m);                     \
    m = fb_max<typename F::LB>(m);                     \
  }
  ISR_FBATCH_SHAPES(FB_LDS)
#undef FB_LDS
  return (m + 255) & ~size_t(255);
}

template <int PREC>
int fbatch_resident_prec(size_t lds_bytes) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_fbatch<PREC>, 256, lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace isr
