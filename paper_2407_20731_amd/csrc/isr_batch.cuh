// One persistent launch for a whole batch of snapshots (orders 5, 7, 9).
//
// Work items live in one global queue, claimed in order through a ticket
// counter.  The queue is phase-major:
//   sample pass, sample select, pass 1, select 1, candidate pass,
//   refine/select levels 2..6, pass 3 (one tile per item), finalize
// and each phase holds the items of every (snapshot, component) pair.  An item
// waits (bounded spin) only on completion counters of EARLIER phases of its own
// pair, whose items hold smaller tickets and so were claimed by workgroups that
// are already running and never wait on later tickets: progress needs no
// co-residency.  Snapshots of different sizes and orders are load balanced
// through the shared queue, and phases of different snapshots overlap.
#pragma once

#include "isr_passes.cuh"
#include "isr_selbody.cuh"

namespace isr {

DEV u32 ld_acq32(const u32* p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT); }
DEV void add_rel32(u32* p, u32 v) { __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }

DEV bool wait_count(const u32* p, u32 target) {
  if (target == 0) return true;
  for (int spins = 0; spins < SPIN_LIMIT; ++spins) {
    if (ld_acq32(p) >= target) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

DEV long long items_of(const BatchCtl& B, int ph, int q) {
  const long long* row = B.items + (size_t)ph * (B.npairs + 1);
  return row[q + 1] - row[q];
}

#define ISR_BATCH_ORDERS(X) X(5) X(7) X(9)

template <int PREC>
__global__ __launch_bounds__(256) void k_batch(BatchCtl B) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ long long tk_s;
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  const long long total = B.phase_off[NPH];
  int p3_pair = -1;
  u32 p3_pending = 0;
  bool p3_first = true;
  for (;;) {
    __syncthreads();
    if (tid == 0) tk_s = (long long)atomicAdd(B.ticket, 1ull);
    __syncthreads();
    const long long tk = tk_s;
    int ph = NPH, q = 0;
    long long k = 0;
    if (tk < total) {
      ph = 0;
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
      q = lo;
      k = x - row[q];
    }
    // a run of pass-3 tiles of one pair ends: flush its error histogram, then
    // count the tiles as done
    if (p3_pair >= 0 && !(ph == PH_P3 && q == p3_pair)) {
      const Job& jp = B.jobs[B.pair_snap[p3_pair]];
      const int cp = B.pair_comp[p3_pair];
      switch (jp.order) {
#define FLUSH(NN)                                                                              \
  case NN: {                                                                                   \
    Pass3Lds<NN, PREC>& L = *reinterpret_cast<Pass3Lds<NN, PREC>*>(lds);                       \
    lh_flush(L.hR, jp.histR + (size_t)cp * HBINS, tid, 256);                                   \
    break;                                                                                     \
  }
        ISR_BATCH_ORDERS(FLUSH)
#undef FLUSH
      }
      __syncthreads();
      if (tid == 0) add_rel32(&B.done[(size_t)PH_P3 * B.npairs + p3_pair], p3_pending);
      p3_pair = -1;
      p3_pending = 0;
    }
    if (ph == NPH) break;
    const int snap = B.pair_snap[q], comp = B.pair_comp[q];
    const Job& j = B.jobs[snap];
    // dependencies: every item of the previous phase of this pair (pass 3: the
    // final select of every component of the snapshot, for the value offsets)
    if (tid == 0) {
      bool ok = true;
      if (ph == PH_P3) {
        const int q0 = q - comp;
        for (int cc = 0; cc < j.ncomp && ok; ++cc)
          ok = wait_count(&B.done[(size_t)PH_S6 * B.npairs + q0 + cc], (u32)items_of(B, PH_S6, q0 + cc));
      } else if (ph > 0) {
        ok = wait_count(&B.done[(size_t)(ph - 1) * B.npairs + q], (u32)items_of(B, ph - 1, q));
      }
      ok_s = ok;
      if (!ok) atomicOr(B.err, 1);
    }
    __syncthreads();
    if (!ok_s) {
      // a dependency never completed (cannot happen): skip the work, keep draining
      if (tid == 0 && ph != PH_P3) add_rel32(&B.done[(size_t)ph * B.npairs + q], 1u);
      continue;
    }
    const long long nk = items_of(B, ph, q);
    if (ph == PH_P0 || ph == PH_P1 || ph == PH_P2) {
      const int sample = ph == PH_P0;
      const long long tstep = sample ? j.sample_stride : 1;
      switch (j.order) {
#define PASS12(NN)                                                                                   \
  case NN:                                                                                           \
    if (ph == PH_P2)                                                                                 \
      pass2_body<NN, PREC>(j, comp, k, nk, *reinterpret_cast<Pass2Lds<NN, PREC>*>(lds));             \
    else                                                                                             \
      pass1_body<NN, PREC>(j, comp, k * tstep, nk * tstep, sample, *reinterpret_cast<Pass1Lds<NN, PREC>*>(lds)); \
    break;
        ISR_BATCH_ORDERS(PASS12)
#undef PASS12
      }
    } else if (ph == PH_S0 || ph == PH_S1) {
      if (tid < 64) select1_body(j, comp, ph == PH_S0);
    } else if (ph == PH_P3) {
      switch (j.order) {
#define PASS3(NN)                                                                              \
  case NN: {                                                                                   \
    typedef typename XfSel<NN, PREC>::type X;                                                  \
    Pass3Lds<NN, PREC>& L = *reinterpret_cast<Pass3Lds<NN, PREC>*>(lds);                       \
    typename X::Regs rg;                                                                       \
    if (p3_pair != q) {                                                                        \
      lh_init(L.hR, tid, 256);                                                                 \
      p3_first = true;                                                                         \
      p3_pair = q;                                                                             \
    }                                                                                          \
    X::init(L.sm, rg, j.tab, tid, 256);                                                        \
    __syncthreads();                                                                           \
    pass3_tile<NN, PREC>(j, comp, k, L, rg, p3_first);                                         \
    break;                                                                                     \
  }
        ISR_BATCH_ORDERS(PASS3)
#undef PASS3
      }
      ++p3_pending;
      continue;
    } else if (ph == PH_FIN) {
      if (tid < 64) finalize_body(j, comp);
    } else {
      // refine level L = 2 + (ph - PH_R2) / 2 (R phases), select level (S phases)
      const int L = 2 + (ph - PH_R2) / 2;
      if (((ph - PH_R2) & 1) == 0)
        refine_body(j, comp, L, reinterpret_cast<u64(*)[2]>(lds), (u64)k, (u64)nk);
      else
        select_body(j, comp, L, *reinterpret_cast<SelLds*>(lds));
    }
    __syncthreads();
    if (tid == 0) add_rel32(&B.done[(size_t)ph * B.npairs + q], 1u);
  }
}

template <int PREC>
hipError_t launch_batch_prec(const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_batch<PREC>, dim3(grid), dim3(256), lds_bytes, s, B);
  return hipGetLastError();
}

template <int PREC>
size_t batch_lds_prec() {
  size_t m = sizeof(u64) * RBINS * 2;
  m = m > sizeof(SelLds) ? m : sizeof(SelLds);
#define SZ(NN)                                                              \
  m = m > sizeof(Pass1Lds<NN, PREC>) ? m : sizeof(Pass1Lds<NN, PREC>);      \
  m = m > sizeof(Pass2Lds<NN, PREC>) ? m : sizeof(Pass2Lds<NN, PREC>);      \
  m = m > sizeof(Pass3Lds<NN, PREC>) ? m : sizeof(Pass3Lds<NN, PREC>);
  ISR_BATCH_ORDERS(SZ)
#undef SZ
  return (m + 255) & ~size_t(255);
}

template <int PREC>
int batch_resident_prec(size_t lds_bytes) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_batch<PREC>, 256, lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace isr
