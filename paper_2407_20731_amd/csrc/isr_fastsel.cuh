// Order-independent kernels of the streaming path as device bodies, so that
// the per-phase launches (isr_select.hip) and the persistent batch launch
// (isr_fbatch.cuh) run the same code.  A body takes the component, the index
// of its (virtual) workgroup and their count in place of blockIdx / gridDim;
// every thread of the workgroup calls it.
#pragma once

#include "isr_selbody.cuh"
#include "isr_xsum.cuh"

namespace isr {

// refine level L over the candidate lists, then (last workgroup of the
// component) the level-L selection
struct RefselLds {
  union {
    u64 h[RBINS][2];
    SelLds S;
  } U;
  int last;
};

DEV void refsel_body(const Job& j, int comp, int L, int vb, int nvb, RefselLds& X) {
  if (j.st[comp].resolved) return;
  refine_body(j, comp, L, X.U.h, vb, nvb);
  if (!last_block(j.done + (D_REFSEL + L) * 8 + comp, &X.last, nvb)) return;
  select_body(j, comp, L, X.U.S);
}

// ---- streaming path: exact window bins, exact totals, level-1 selection ------
// Every workgroup adds the significands of its share of list 0 (the window
// energies) to the window bins; workgroup 0 turns the per-workgroup integer
// sums of pass A into exact bins (norm terms anywhere, energies below the
// window in bins below it) and puts the count of energies above the window
// into bin win_hi; the last workgroup runs the level-1 selection.
struct GatherLds {
  u64 red[4][9];
  __int128 r7[4][7], r9[4][9];
  int last;
};

DEV void gather_body(const Job& j, int comp, int vb, int nvb, GatherLds& X) {
  u64(&red)[4][9] = X.red;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const int wlo = st->win_lo, whi = st->win_hi;
  HistBin* gE = j.histE + (size_t)comp * HBINS;
  HistBin* gN = j.histN + (size_t)comp * HBINS;
  const u64* list = list_ptr(j, comp, 0);
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  u64 acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // (cnt, lo, hi) of the three window bins
  for (u64 i = (u64)vb * 256 + tid; i < nl; i += (u64)nvb * 256) {
    const u64 key = list[i];
    const int k = (int)(key >> 52) - wlo;  // 0..2; window bins are >= 1 (normal numbers)
    const u64 sig = (key & M52) | (1ull << 52);
    for (int b = 0; b < 3; ++b) {
      if (b == k) {
        acc[3 * b] += 1ull;
        acc[3 * b + 1] += sig & M21;
        acc[3 * b + 2] += sig >> 21;
      }
    }
  }
  for (int k = 0; k < 9; ++k) {
    const u64 w = wave_sum64(acc[k]);
    if (lane == 0) red[wv][k] = w;
  }
  __syncthreads();
  // per-workgroup partials (no contended atomics); the last workgroup adds them
  if (tid < 9) j.gslot[((size_t)comp * GATHER_GMAX + vb) * 16 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  if (vb == 0) {
    // totals of pass A's workgroup sums: fields 0..2 norm, 3..5 energy, 6 count
    __int128 T[7];
    block_totals<7>(j.slotsA + (size_t)comp * j.gA * 8, j.gA, 8, T, X.r7, tid);
    if (tid == 0) {
      __int128 K[3];
      for (int k = 0; k < 3; ++k) K[k] = T[k];
      emit_total(gN, K, st->xm_norm, j.xh, -1);
      for (int k = 0; k < 3; ++k) K[k] = T[3 + k];
      if (wlo < whi) emit_total(gE, K, wlo - 1023, j.xh, wlo - 1);
      const u64 above = (u64)T[6];
      if (above) atomicAdd(&gE[whi].cnt, above);
    }
  }
  if (!last_block(j.done + D_GATHER * 8 + comp, &X.last, nvb)) return;
  __int128 T9[9];
  block_totals<9>((const long long*)j.gslot + (size_t)comp * GATHER_GMAX * 16, nvb, 16, T9, X.r9, tid);
  for (int k = 0; k < 9; ++k) {
    const u64 w = (u64)T9[k];
    const int b = wlo + k / 3;
    if (tid == 0 && w && b < whi) {
      if (k % 3 == 0) atomicAdd(&gE[b].cnt, w);
      if (k % 3 == 1) atomicAdd(&gE[b].lo, w);
      if (k % 3 == 2) atomicAdd(&gE[b].hi, w);
    }
  }
  __threadfence();
  __syncthreads();
  if (tid < 64) select1_body(j, comp, 0);
  __syncthreads();
  if (tid == 0) {
    // bound on the error terms of pass B: a little above the budget, or, when
    // everything is kept, a little above the rounding level of the transforms
    int m;
    if (st->B > 0.0) {
      m = ilogb(st->B) + 6;
    } else {
      const int eu = st->U2 > 0.0 ? ilogb(st->U2) : XM_MIN;
      m = eu - (j.precision == 0 ? 80 : 30);
    }
    st->xm_err = m < XM_MIN ? XM_MIN : (m > XM_MAX ? XM_MAX : m);
  }
}

// Per-element kept counts: pass A stored the count of energies above the
// window; every window entry of list 0 at or above tau adds one.
DEV void count_body(const Job& j, int comp, int vb, int nvb) {
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  u32* cnt = j.cnt + (size_t)comp * j.n_elem;
  const u64 tk = dbits(st->tau);
  const u64* list = list_ptr(j, comp, 0);
  const u32* lidx = j.lidx + (size_t)comp * j.list_cap;
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  for (u64 i = (u64)vb * 256 + tid; i < nl; i += (u64)nvb * 256)
    if (list[i] >= tk) atomicAdd(&cnt[lidx[i]], 1u);
}

// Element offsets from the counts, in two steps over chunks of SCAN_CHUNK
// elements: chunk sums (the last workgroup turns them into chunk offsets and
// checks the total against the selected kept count), then a local scan of
// every chunk.
DEV u64 block_excl_scan(u64 v, u64* part, int tid, u64* total) {
  part[tid] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const u64 o = tid >= d ? part[tid - d] : 0ull;
    __syncthreads();
    part[tid] += o;
    __syncthreads();
  }
  const u64 incl = part[tid];
  *total = part[255];
  __syncthreads();
  return incl - v;
}

struct ScanLds {
  u64 part[256];
  int last;
};

DEV void scan1_body(const Job& j, int comp, int vb, int nvb, ScanLds& X) {
  u64* part = X.part;
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const long long E = j.n_elem;
  const u32* cnt = j.cnt + (size_t)comp * E;
  const long long nch = (E + SCAN_CHUNK - 1) / SCAN_CHUNK;
  u64* coff = j.chunk + (size_t)comp * j.nchunk;
  for (long long c = vb; c < nch; c += nvb) {
    u64 v = 0;
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
      const long long e = c * SCAN_CHUNK + k * 256 + tid;
      if (e < E) v += cnt[e];
    }
    u64 tot;
    (void)block_excl_scan(v, part, tid, &tot);
    if (tid == 0) coff[c] = tot;
  }
  if (!last_block(j.done + D_COUNT * 8 + comp, &X.last, nvb)) return;
  // chunk sums -> exclusive chunk offsets (in place), total check
  u64 run = 0;
  for (long long c0 = 0; c0 < nch; c0 += 256) {
    const long long c = c0 + tid;
    const u64 v = c < nch ? coff[c] : 0ull;
    u64 tot;
    const u64 ex = block_excl_scan(v, part, tid, &tot);
    if (c < nch) coff[c] = run + ex;
    run += tot;
  }
  if (tid == 0) {
    j.elem_ptr[(size_t)comp * (E + 1) + E] = run;
    if (run != st->kept) atomicOr(&st->flags, ST_LIST);
  }
}

DEV void scan2_body(const Job& j, int comp, int vb, int nvb, ScanLds& X) {
  u64* part = X.part;
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const long long E = j.n_elem;
  const u32* cnt = j.cnt + (size_t)comp * E;
  const long long nch = (E + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const u64* coff = j.chunk + (size_t)comp * j.nchunk;
  u64* eptr = j.elem_ptr + (size_t)comp * (E + 1);
  for (long long c = vb; c < nch; c += nvb) {
    // thread t owns elements c*CHUNK + 4t .. 4t+3
    const long long e0 = c * SCAN_CHUNK + 4 * tid;
    u32 v[4];
    u64 sum = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = e0 + k < E ? cnt[e0 + k] : 0u;
      sum += v[k];
    }
    u64 tot;
    u64 run = coff[c] + block_excl_scan(sum, part, tid, &tot);
    for (int k = 0; k < 4; ++k) {
      if (e0 + k < E) eptr[e0 + k] = run;
      run += v[k];
    }
  }
}


}  // namespace isr
