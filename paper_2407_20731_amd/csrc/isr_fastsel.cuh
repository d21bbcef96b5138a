// Order-independent kernels of the streaming path as device bodies, so that
// the per-phase launches (isr_select.hip) and the persistent batch launch
// (isr_fbatch.cuh) run the same code.  A body takes the component, the index
// of its (virtual) workgroup and their count in place of blockIdx / gridDim;
// every thread of the workgroup calls it.
//
// A phase whose result needs every workgroup's share (a selection, a total)
// ends in a tail that runs once per component.  The per-phase launches run
// the tail as a kernel of its own after the phase (the kernel boundary makes
// the shares visible); the persistent batch, which has no such boundary, runs
// it in the last workgroup to finish (`tail` = true), behind a device-scope
// fence in every workgroup.  The fence writes back the L2 cache of the
// workgroup's XCD, which costs tens of microseconds over a few hundred
// workgroups, so the per-phase launches avoid it.
#pragma once

#include "isr_selbody.cuh"
#include "isr_xsum.cuh"

namespace isr {

// One wave per component: window [b - 1, b + 2) around the bin b where the
// rounded cumulative sampled energy first exceeds tol^2 * (sampled U2), and
// the norm-term bound 2^(largest sampled exponent + 8).
DEV void select_sample_body(const Job& j, int comp) {
  const int lane = lane_id();
  CompState* st = j.st + comp;
  const HistBin* H = j.histEs + (size_t)comp * HBINS;
  if (lane == 0) {
    const int mx = st->samp_maxe;  // biased; 0 when every sampled term is 0
    int m = mx - 1023 + 8;
    m = m < XM_MIN ? XM_MIN : (m > XM_MAX ? XM_MAX : m);
    st->xm_norm = m;
    st->win_mode = 1;
  }
  const double tol = j.tol;
  if (tol < 0.0) {  // keep everything: no window, every energy counts as "above"
    if (lane == 0) st->win_lo = st->win_hi = 0;
    return;
  }
  const double B = ((tol * tol) * st->samp_u2) * j.cut_scale;
  // (the sampled bins hold rounded sums only: one atomic per bin and
  // workgroup, and a bin of positive energies has a positive sum)
  double cs = 0.0;
  for (int k = 0; k < 32; ++k) {
    const int b = 32 * lane + k;
    if (b < HBINS - 1) cs += __longlong_as_double((long long)H[b].lo);
  }
  double incl = cs;
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  const u64 over = ballot(incl > B);
  const u64 nonempty = ballot(cs > 0.0);
  int bstar = -1;
  if (over) {
    const int fl = __ffsll((long long)over) - 1;
    double cum = __shfl(incl - cs, fl);
    for (int k = 0; k < 32; ++k) {
      const int b = 32 * fl + k;
      if (b >= HBINS - 1) break;
      cum += __longlong_as_double((long long)H[b].lo);
      if (cum > B) {
        bstar = b;
        break;
      }
    }
  } else if (nonempty) {
    // every sampled energy fits the budget: the top bin (tau is likely +inf,
    // which the general pipeline handles)
    const int fl = 63 - __clzll((long long)nonempty);
    for (int k = 31; k >= 0; --k) {
      const int b = 32 * fl + k;
      if (b < HBINS - 1 && __longlong_as_double((long long)H[b].lo) > 0.0) {
        bstar = b;
        break;
      }
    }
  }
  if (lane == 0) {
    const int wl = bstar - 1 < 1 ? 1 : bstar - 1;
    const int wh = bstar + 2 > HBINS - 2 ? HBINS - 2 : bstar + 2;
    if (bstar < 0 || wl - 1023 < XM_MIN || wl >= wh) {
      st->flags |= ST_MISS;
      st->resolved = 1;
    } else {
      st->win_lo = wl;
      st->win_hi = wh;
    }
  }
}

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
// energies) to the window bins (integer sums: exact in any order); workgroup 0
// also turns the per-workgroup integer sums of pass A into exact bins (norm
// terms anywhere, energies below the window in bins below it) and puts the
// count of energies above the window into bin win_hi.  The tail runs the
// level-1 selection.
struct GatherLds {
  u64 red[4][9];
  __int128 r7[4][7];
  int last;
};

DEV void gather_tail(const Job& j, int comp) {
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
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

DEV void gather_body(const Job& j, int comp, int vb, int nvb, GatherLds& X, bool tail) {
  u64(&red)[4][9] = X.red;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const int wlo = st->win_lo, whi = st->win_hi;
  HistBin* gE = j.histE + (size_t)comp * HBINS;
  if (vb == 0) {
    // totals of pass A's workgroup sums: fields 0..2 norm, 3..5 energy, 6 count
    __int128 T[7];
    block_totals<7>(j.slotsA + (size_t)comp * j.gA * 8, j.gA, 8, T, X.r7, tid);
    if (tid == 0) {
      __int128 K[3];
      for (int k = 0; k < 3; ++k) K[k] = T[k];
      emit_total(j.histN + (size_t)comp * HBINS, K, st->xm_norm, j.xh, -1);
      for (int k = 0; k < 3; ++k) K[k] = T[3 + k];
      if (wlo < whi) emit_total(gE, K, wlo - 1023, j.xh, wlo - 1);
      const u64 above = (u64)T[6];
      if (above) atomicAdd(&gE[whi].cnt, above);
    }
  }
  const u64* list = list_ptr(j, comp, 0);
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  u64 acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // (cnt, lo, hi) of the three window bins
  // sixteen entries per lane per step, loaded before any is used
  constexpr int U = 16;
  const u64 stride = (u64)nvb * 256;
  for (u64 i0 = (u64)vb * 256 + tid; i0 < nl; i0 += U * stride) {
    u64 keys[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u64 i = i0 + u * stride;
      keys[u] = i < nl ? list[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * stride >= nl) continue;
      const u64 key = keys[u];
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
  }
  for (int k = 0; k < 9; ++k) {
    const u64 w = wave_sum64(acc[k]);
    if (lane == 0) red[wv][k] = w;
  }
  __syncthreads();
  if (tid < 9) {
    const u64 w = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    const int b = wlo + tid / 3;
    if (w && b < whi) {
      HistBin& h = gE[b];
      atomicAdd(tid % 3 == 0 ? &h.cnt : (tid % 3 == 1 ? &h.lo : &h.hi), w);
    }
  }
  if (!tail || !last_block(j.done + D_GATHER * 8 + comp, &X.last, nvb)) return;
  gather_tail(j, comp);
}

// Per-element kept counts: pass A stored the count of energies above the
// window; every window entry of list 0 at or above tau adds one.
DEV void count_body(const Job& j, int comp, int vb, int nvb) {
  const int tid = threadIdx.x, lane = tid & 63;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  u32* cnt = j.cnt + (size_t)comp * j.n_elem;
  const u64 tk = dbits(st->tau);
  const u64* list = list_ptr(j, comp, 0);
  const u32* lidx = j.lidx + (size_t)comp * j.list_cap;
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  constexpr int U = 4;
  const u64 stride = (u64)nvb * 256;
  // the trip count is the same for every lane of a wave (ballots inside)
  const u64 nl_r = (nl + 63) & ~63ull;
  for (u64 i0 = (u64)vb * 256 + tid; i0 < nl_r; i0 += U * stride) {
    u64 keys[U];
    u32 idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u64 i = i0 + u * stride;
      keys[u] = i < nl ? list[i] : 0ull;
      idx[u] = i < nl ? lidx[i] : 0u;
    }
    // list entries of one element sit close together: one atomic per
    // distinct element of the wave (leader = lowest lane) instead of one per
    // entry
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bool act = i0 + u * stride < nl && keys[u] >= tk;
      u64 m = ballot(act);
      while (m) {
        const int l = __ffsll((long long)m) - 1;
        const u32 el = (u32)__shfl((int)idx[u], l);
        const u64 same = ballot(act && idx[u] == el);
        if (lane == l) atomicAdd(&cnt[el], (u32)__popcll(same));
        act = act && idx[u] != el;
        m &= ~same;
      }
    }
  }
}

// Element offsets from the counts, in two steps over chunks of SCAN_CHUNK
// elements: chunk sums, then a local scan of every chunk on top of the sum of
// the chunk sums before it (the last chunk's workgroup also writes the total
// and checks it against the selected kept count).
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
    // the chunk's offset: the sum of the chunk sums before it
    u64 pre = 0;
    for (long long k = tid; k < c; k += 256) pre += coff[k];
    u64 base;
    (void)block_excl_scan(pre, part, tid, &base);
    // thread t owns elements c*CHUNK + 4t .. 4t+3
    const long long e0 = c * SCAN_CHUNK + 4 * tid;
    u32 v[4];
    u64 sum = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = e0 + k < E ? cnt[e0 + k] : 0u;
      sum += v[k];
    }
    u64 tot;
    u64 run = base + block_excl_scan(sum, part, tid, &tot);
    for (int k = 0; k < 4; ++k) {
      if (e0 + k < E) eptr[e0 + k] = run;
      run += v[k];
    }
    if (c == nch - 1 && tid == 0) {
      eptr[E] = base + tot;
      if (base + tot != st->kept) atomicOr(&st->flags, ST_LIST);
    }
  }
}

// Pass B's tail: the component's error total from the per-workgroup integer
// sums, then its final statistics.
DEV void passB_tail(const Job& j, int comp, __int128 (*r3)[3]) {
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const XParm PR = xparm(st->xm_err, j.xh);
  __int128 K[3];
  block_totals<3>(j.slotsB + (size_t)comp * j.gB * 4, j.gB, 4, K, r3, tid);
  if (tid == 0) emit_total(j.histR + (size_t)comp * HBINS, K, PR.m, PR.h, -1);
  __threadfence();
  __syncthreads();
  if (tid < 64) finalize_body(j, comp);
}

}  // namespace isr
