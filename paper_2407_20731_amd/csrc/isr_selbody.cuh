// Threshold-selection bodies (device functions), shared by the per-phase
// kernels (isr_select.hip) and the persistent batch kernel (isr_batch.cuh).
// The threshold rule (arXiv 2407.20731, Sec. IV-B reading): tau is the largest
// energy value v whose dropped energy S(v) = RN(exact sum of energies < v)
// does not exceed B = (tol*tol)*U2.
#pragma once

#include "isr.h"
#include "isr_common.cuh"

namespace isr {

// --------------------------------------------------------------------------
// select, level 1 (one wave per component): U2, B, the slack integer
// Tint = largest X-unit sum whose round-to-nearest is <= B, and the boundary
// exponent bin b*: the last non-empty bin whose exclusive prefix sum is <= Tint.

// With sample = 1 the same walk runs on the histograms of the sampled tiles
// and only records the window of exponent bins [b - 1, b + 2) that pass 1
// then copies to the candidate list; with sample = 0 it decides whether the
// true boundary bin fell inside that window (else the candidate pass runs).
// Run by one whole wave.
DEV void select1_body(const Job& j, int comp, int sample) {
  const int lane = lane_id();
  CompState* st = j.st + comp;
  const HistBin* HN = (sample ? j.histNs : j.histN) + (size_t)comp * HBINS;
  const HistBin* HE = (sample ? j.histEs : j.histE) + (size_t)comp * HBINS;
  const double tol = j.tol;
  int flags = 0;
  if (HN[HBINS - 1].cnt) flags |= ST_NONFINITE;
  if (HE[HBINS - 1].cnt) flags |= ST_OVERFLOW;
  u64 U = hist_total(HN);
  const double U2 = wb_round(U);
  if (sample) {
    if (tol < 0.0) return;
  } else if (lane == 0) {
    const int nn = j.order + 1;
    st->U2 = U2;
    st->tol = tol;
    st->n_values = (u64)j.n_elem * (u64)(nn * nn * nn);
    st->flags |= flags;
  }
  if (tol < 0.0) {  // keep everything
    if (lane == 0) {
      st->B = 0.0;
      st->tau = 0.0;
      st->kept = st->n_values;
      st->dropped = 0.0;
      st->bstar = -1;
      st->resolved = 1;
      st->level = 1;
    }
    return;
  }
  double B = (tol * tol) * U2;
  if (j.cut_scale != 1.0) B = B * j.cut_scale;  // a share of the budget left to a later stage
  // MFMA paths: the measured error differs from the dropped energy by the
  // transform error (about 1e-5 relative in FP32-split BF16 at tol 1e-3), so
  // they select against a budget that much smaller and rarely need a repair
  if (j.precision == ISR_PREC_BF16)
    B = B * (1.0 - 0x1p-10);
  else if (j.precision == ISR_PREC_FP32)
    B = B * (1.0 - 0x1p-17);
  if (!sample && comp < 8 && j.Bov[comp] >= 0.0) B = j.Bov[comp];
  // Tint = X(B) + half ulp(B) - (sig(B) odd)
  const u64 bb = dbits(B);
  const int EB = (int)(bb >> 52);
  const u64 sigB = (bb & M52) | (EB ? (1ull << 52) : 0ull);
  const int sB = EB > 1 ? EB : 1;
  u64 Tw = 0;
  const bool Binf = EB == 2047;
  if (!Binf) {
    wb_add(Tw, part_at(sigB, 0ull, sB));
    wb_add(Tw, part_at(1ull, 0ull, sB - 1));
    if (sigB & 1ull) wb_sub(Tw, part_at(1ull, 0ull, 0));
  }
  // walk the energy bins
  u64 clo, chi, ccnt;
  int base;
  chunk32(HE, clo, chi, ccnt, base);
  u64 R = Tw, P = 0ull;
  int bstar = -1, lcross = 64;
  u64 cross_cnt = 0ull;  // this lane's bin of the crossing chunk: its count
  bool found = false;
  for (int l = 0; l < 64 && !Binf; ++l) {
    const u64 cc = bcast64(ccnt, l);
    if (cc == 0ull) continue;
    const u64 cl = bcast64(clo, l), ch = bcast64(chi, l);
    const int bl = l == 0 ? 1 : 32 * l;
    u64 tmp = R;
    wb_sub(tmp, part_at(cl, ch, bl));
    if (!wb_neg(tmp)) {
      R = tmp;
      wb_add(P, part_at(cl, ch, bl));
      continue;
    }
    // the crossing chunk, one bin per lane (loads in parallel, then broadcast)
    const int mybin = 32 * l + lane;
    const HistBin mine = (lane < 32 && mybin < HBINS - 1) ? HE[mybin] : HistBin{0ull, 0ull, 0ull};
    lcross = l;
    cross_cnt = mine.cnt;
    for (int k = 0; k < 32; ++k) {
      const int bin = 32 * l + k;
      if (bin >= HBINS - 1) break;
      const HistBin h = {bcast64(mine.cnt, k), bcast64(mine.lo, k), bcast64(mine.hi, k)};
      if (h.cnt == 0ull) continue;
      bstar = bin;
      const u128 sb = bin_sum(h);
      const u64 sl = (u64)sb, sh = (u64)(sb >> 64);
      const int s = bin > 1 ? bin : 1;
      u64 t2 = R;
      wb_sub(t2, part_at(sl, sh, s));
      if (wb_neg(t2)) break;
      R = t2;
      wb_add(P, part_at(sl, sh, s));
    }
    found = true;
    break;
  }
  if (!sample && st->win_mode) {
    // the streaming pass kept exact sums only inside the window: a boundary
    // outside it (or none at all) sends the request to the general pipeline
    const bool hit = found && bstar >= st->win_lo && bstar < st->win_hi;
    if (!hit) {
      if (lane == 0) {
        st->flags |= ST_MISS;
        st->resolved = 1;
      }
      return;
    }
  }
  if (sample) {
    if (lane == 0 && found) {
      st->win_lo = bstar > 0 ? bstar - 1 : 0;
      st->win_hi = bstar + 2 < HBINS - 1 ? bstar + 2 : HBINS - 1;
    }
    return;
  }
  if (!found) {  // every energy can be dropped: tau = +inf
    double dropped = 0.0;
    if (Binf) {
      u64 tot = hist_total(HE);
      dropped = wb_round(tot);
    } else {
      dropped = wb_round(P);
    }
    if (lane == 0) {
      st->B = B;
      st->tau = __builtin_inf();
      st->kept = 0ull;
      st->dropped = dropped;
      st->bstar = -1;
      st->resolved = 1;
      st->level = 1;
    }
    return;
  }
  // counts above b*: the chunks above the crossing one, and the crossing
  // chunk's bins above b* (bin HBINS - 1 is in neither)
  u64 above = (lane > lcross ? ccnt : 0ull) + (lane < 32 && 32 * lcross + lane > bstar ? cross_cnt : 0ull);
  above = wave_sum64(above);
  const int s = bstar > 1 ? bstar : 1;
  u64 rlo, rhi;
  bool sat;
  wb_extract128(R, s, rlo, rhi, sat);
  if (sat) rlo = rhi = ~0ull;
  st->P1[lane] = P;
  if (lane == 0) {
    st->B = B;
    st->bstar = bstar;
    st->kept_above = above;
    st->cur_count = HE[bstar].cnt;
    st->key_prefix = (u64)bstar << 52;
    st->key_mask = 0x7FFull << 52;
    st->r_lo = rlo;
    st->r_hi = rhi;
    st->w_lo = 0ull;
    st->w_hi = 0ull;
    st->level = 1;
    st->resolved = 0;
    // pass 1 captured the window [win_lo, win_hi); outside it, pass 2 gathers
    // the boundary bin into a fresh list 0
    const bool hit = bstar >= st->win_lo && bstar < st->win_hi;
    st->need_pass2 = hit ? 0 : 1;
    st->list0_exact = hit ? 0 : 1;
    if (!hit) st->list_count[0] = 0ull;
  }
}

// --------------------------------------------------------------------------
// refine, level L in 2..6: histogram of the next fraction bits of the listed
// energies that match the current prefix; for L >= 3 the matching keys are
// also copied to the other list.

// List 0 (the candidates of the boundary bin or window) is only read, by
// levels 2 and 3; levels 3..6 copy the members of the current sub-bin to
// lists 1, 2, 1, 2, so list 0 stays whole for the per-element kept counts.
DEV int list_out(int L) { return (L & 1) ? 1 : 2; }
DEV int list_in(int L) { return L <= 3 ? 0 : 3 - list_out(L); }
DEV int list_members(int L) { return L == 2 ? 0 : list_out(L); }

// Worker `item` of `nitems` handles list entries item*256 + tid + k*nitems*256
// (blockDim must be 256).
DEV void refine_body(const Job& j, int comp, int L, u64 (*h)[2], u64 item, u64 nitems) {
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->resolved) return;
  __syncthreads();
  const int nb = 1 << level_bits(L), sh = level_shift(L);
  const u64 fmask = (u64)(nb - 1);
  for (int k = tid; k < nb; k += 256) h[k][0] = h[k][1] = 0ull;
  __syncthreads();
  const int li = list_in(L);
  const u64* in = list_ptr(j, comp, li);
  const u64 nin = st->list_count[li] < list_capk(j, li) ? st->list_count[li] : list_capk(j, li);
  const u64 prefix = st->key_prefix, mask = st->key_mask;
  const int bstar = st->bstar;
  const u64 implicit = bstar ? (1ull << 52) : 0ull;
  const int lo_idx = L >= 3 ? list_out(L) : 0;
  u64* out = list_ptr(j, comp, lo_idx);
  const u64 stride = nitems * 256;
  // the loop trip count is the same for every lane of a wave (ballots inside)
  const u64 nin_r = (nin + 63) & ~63ull;
  // sixteen entries per lane per step, loaded before any is used (the lists
  // run to millions of entries: more loads in flight per lane)
  constexpr int U = 16;
  for (u64 i0 = item * 256 + tid; i0 < nin_r; i0 += U * stride) {
    u64 keys[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u64 i = i0 + u * stride;
      keys[u] = i < nin ? in[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u64 i = i0 + u * stride;
      const u64 key = keys[u];
      const bool m = i < nin && (key & mask) == prefix;
      if (m) {
        const u64 sig = (key & M52) | implicit;
        const int sb = (int)((key >> sh) & fmask);
        atomicAdd(&h[sb][0], (1ull << 43) + (sig & M21));
        atomicAdd(&h[sb][1], sig >> 21);
      }
      // (i < nin_r is the same for every lane of a wave: ballots inside)
      if (L >= 3 && i < nin_r) list_append(out, &st->list_count[lo_idx], list_capk(j, lo_idx), m, key, &st->flags);
    }
  }
  __syncthreads();
  HistBin* g = j.histL + ((size_t)(L - 2) * j.ncomp + comp) * RBINS;
  for (int k = tid; k < nb; k += 256) {
    const u64 w0 = h[k][0], w1 = h[k][1];
    if (w0 | w1) global_bin_add(g, k, w0 >> 43, w0 & M43, w1);
  }
  __syncthreads();
}


// Resolve tau among <= CAP listed members of the current sub-bin by sorting
// them and scanning their significands in ascending order.
DEV void resolve_sorted(const Job& j, CompState* st, int comp, int ml, int L, u64* keys, u64* slo, u64* shi,
                        int* best) {
  const int tid = threadIdx.x;
  const u64* list = list_ptr(j, comp, ml);
  const u64 lc = st->list_count[ml];
  const int cnt = (int)(lc < (u64)CAP ? lc : (u64)CAP);  // == cur_count unless a list overflowed
  int np = 1;
  while (np < cnt) np <<= 1;
  for (int i = tid; i < np; i += 256) keys[i] = i < cnt ? list[i] : ~0ull;
  if (tid == 0) *best = 0;
  __syncthreads();
  for (int k = 2; k <= np; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < np; i += 256) {
        const int ixj = i ^ jj;
        if (ixj > i) {
          const u64 x = keys[i], y = keys[ixj];
          const bool asc = (i & k) == 0;
          if ((x > y) == asc) {
            keys[i] = y;
            keys[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const u64 implicit = st->bstar ? (1ull << 52) : 0ull;
  const int per = (np + 255) / 256;
  const int i0 = tid * per;
  u128 run = 0;
  for (int k = 0; k < per; ++k) {
    const int i = i0 + k;
    if (i < cnt) run += (u128)((keys[i] & M52) | implicit);
  }
  // inclusive scan of the 256 per-thread sums (Hillis-Steele in LDS)
  u128 incl = run;
  for (int d = 1; d < 256; d <<= 1) {
    slo[tid] = (u64)incl;
    shi[tid] = (u64)(incl >> 64);
    __syncthreads();
    u128 add = 0;
    if (tid >= d) add = ((u128)shi[tid - d] << 64) | slo[tid - d];
    __syncthreads();
    incl += add;
  }
  const u128 r = ((u128)st->r_hi << 64) | st->r_lo;
  u128 ex = incl - run;
  int mybest = -1;
  u128 myex = 0;
  for (int k = 0; k < per; ++k) {
    const int i = i0 + k;
    if (i >= cnt) break;
    const bool first = i == 0 || keys[i] != keys[i - 1];
    if (first && ex <= r) {
      mybest = i;
      myex = ex;
    }
    ex += (u128)((keys[i] & M52) | implicit);
  }
  if (mybest >= 0) atomicMax(best, mybest);
  __syncthreads();
  const int bi = *best;
  if (mybest >= 0 && mybest == bi) {
    const u128 w = (((u128)st->w_hi << 64) | st->w_lo) + myex;
    st->w_lo = (u64)w;
    st->w_hi = (u64)(w >> 64);
    st->tau = __longlong_as_double((long long)keys[bi]);
    st->kept = st->kept_above + (u64)(cnt - bi);
    st->resolved = 1;
    st->level = L;
    if (lc != st->cur_count) st->flags |= ST_LIST;
  }
}

struct SelLds {
  u64 keys[CAP];
  u64 slo[256], shi[256];
  int best;
};

// blockDim must be 256; the sub-bin walk runs on wave 0.
// One wave walks the NB = 64 PER sub-bins of level L: lane l sums sub-bins
// [PER l, PER l + PER), a 128-bit scan finds the lane whose chunk crosses the
// remaining budget, and that chunk's sub-bins are loaded one per lane and
// walked in registers.  Every load of a step is issued before any is used.
template <int PER>
DEV void select_walk(const Job& j, CompState* st, int comp, int L) {
  const int nb = 1 << level_bits(L), sh = level_shift(L);
  const HistBin* H = j.histL + ((size_t)(L - 2) * j.ncomp + comp) * RBINS;
  const int lane = lane_id();
  u128 cs = 0;
#pragma unroll 8
  for (int k = 0; k < PER; ++k) {
    const int sb = lane * PER + k;
    if (sb < nb) cs += bin_sum(H[sb]);
  }
  // inclusive scan of the lane chunk sums
  u64 ilo = (u64)cs, ihi = (u64)(cs >> 64);
  for (int d = 1; d < 64; d <<= 1) {
    const u64 olo = shfl_up64(ilo, d), ohi = shfl_up64(ihi, d);
    if (lane >= d) {
      const u128 v = (((u128)ihi << 64) | ilo) + (((u128)ohi << 64) | olo);
      ilo = (u64)v;
      ihi = (u64)(v >> 64);
    }
  }
  const u128 r = ((u128)st->r_hi << 64) | st->r_lo;
  const u128 incl = ((u128)ihi << 64) | ilo;
  const u64 over = ballot(incl > r);
  if (over == 0ull) {  // cannot happen: the current bin's total exceeds r
    if (lane == 0) {
      st->flags |= ST_LIST;
      st->tau = __builtin_nan("");
      st->resolved = 1;
    }
    return;
  }
  const int fl = __ffsll((long long)over) - 1;
  u128 excl = 0;
  {
    const u128 myex = incl - cs;
    const u64 elo = bcast64((u64)myex, fl), ehi = bcast64((u64)(myex >> 64), fl);
    excl = ((u128)ehi << 64) | elo;
  }
  // the crossing chunk, one sub-bin per lane, then walked in registers
  const int msb = fl * PER + lane;
  const HistBin mine = (lane < PER && msb < nb) ? H[msb] : HistBin{0ull, 0ull, 0ull};
  int chosen = -1;
  u64 ccnt = 0ull;
  for (int k = 0; k < PER; ++k) {
    const u64 c = bcast64(mine.cnt, k);
    if (c == 0ull) continue;
    const u128 s = (((u128)bcast64(mine.hi, k)) << 21) + (u128)bcast64(mine.lo, k);
    chosen = fl * PER + k;
    ccnt = c;
    if (excl + s > r) break;
    excl += s;
  }
  if (chosen < 0) {  // cannot happen: the crossing chunk is non-empty
    if (lane == 0) {
      st->flags |= ST_LIST;
      st->tau = __builtin_nan("");
      st->resolved = 1;
    }
    return;
  }
  u64 above = 0;
#pragma unroll 8
  for (int k = 0; k < PER; ++k) {
    const int sb = lane * PER + k;
    if (sb < nb && sb > chosen) above += H[sb].cnt;
  }
  above = wave_sum64(above);
  if (lane == 0) {
    const u128 rn = r - excl;
    st->r_lo = (u64)rn;
    st->r_hi = (u64)(rn >> 64);
    const u128 w = (((u128)st->w_hi << 64) | st->w_lo) + excl;
    st->w_lo = (u64)w;
    st->w_hi = (u64)(w >> 64);
    st->kept_above += above;
    st->cur_count = ccnt;
    st->key_prefix |= (u64)chosen << sh;
    st->key_mask |= ((u64)nb - 1ull) << sh;
    st->level = L;
    if (L == NLEV) {  // every bit fixed: the sub-bin is the single value tau
      st->tau = __longlong_as_double((long long)st->key_prefix);
      st->kept = st->kept_above + st->cur_count;
      st->resolved = 1;
    } else {
      st->list_count[list_out(L + 1)] = 0ull;
    }
  }
}

DEV void select_body(const Job& j, int comp, int L, SelLds& S) {
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->resolved) return;
  const int ml = list_members(L);
  __syncthreads();
  if (st->cur_count <= (u64)CAP && (L > 2 || st->list0_exact)) {
    resolve_sorted(j, st, comp, ml, L, S.keys, S.slo, S.shi, &S.best);
    return;
  }
  if (tid >= 64) return;
  // walk the level-L sub-bins with one wave
  if (level_bits(L) == 11)
    select_walk<(1 << 11) / 64>(j, st, comp, L);
  else
    select_walk<((1 << 8) + 63) / 64>(j, st, comp, L);
}

// --------------------------------------------------------------------------
// finalize (one wave per component): err2, rel, dropped energy.

// Run by one whole wave.
DEV void finalize_body(const Job& j, int comp) {
  const int lane = lane_id();
  CompState* st = j.st + comp;
  u64 er = hist_total(j.histR + (size_t)comp * HBINS);
  const double err2 = wb_round(er);
  const double U2 = st->U2;
  const double rel = U2 > 0.0 ? __builtin_sqrt(err2 / U2) : 0.0;
  double dropped = st->dropped;
  if (st->resolved && st->bstar >= 0) {
    u64 P = st->P1[lane];
    const int s = st->bstar > 1 ? st->bstar : 1;
    wb_add(P, part_at(st->w_lo, st->w_hi, s));
    dropped = wb_round(P);
  }
  if (lane == 0) {
    st->err2 = err2;
    st->rel = rel;
    st->dropped = dropped;
    if (!st->resolved) st->flags |= ST_SPIN;
    u64 vo = 0;
    for (int cc = 0; cc < comp; ++cc) vo += j.st[cc].kept;
    j.voff[comp] = vo;
  }
}

}  // namespace isr
