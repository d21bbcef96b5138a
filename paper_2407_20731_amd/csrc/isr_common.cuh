// Device building blocks shared by the kernels: shapes, exact-sum histograms,
// wave-distributed big integers, and the FP64 fixed-order contractions.
#pragma once

#include "isr_internal.h"

namespace isr {

#define DEV __device__ __forceinline__

constexpr u64 M52 = (1ull << 52) - 1;
constexpr u64 M21 = (1ull << 21) - 1;
constexpr u64 M43 = (1ull << 43) - 1;
constexpr u64 M62 = (1ull << 62) - 1;
typedef unsigned __int128 u128;

// ---- element tile shapes --------------------------------------------------
// A workgroup works on EPI elements at a time; one thread per (element,
// pencil) with n^2 pencils per element.
template <int N>
struct Shape {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int EPI = (256 / n2) > 0 ? (256 / n2) : 1;
  static constexpr int ACT = EPI * n2;
  static constexpr int THREADS = ((ACT + 63) / 64) * 64;
  static constexpr int TILE = EPI * n3;
  static constexpr int W = (n3 + 63) / 64;
};

DEV u64 dbits(double v) { return (u64)__double_as_longlong(v); }
DEV int lane_id() { return (int)__lane_id(); }

// ---- wave helpers -----------------------------------------------------------
DEV u64 ballot(bool p) { return (u64)__ballot(p); }
DEV u64 bcast64(u64 v, int src) {
  u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)v, src);
  u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(v >> 32), src);
  return ((u64)hi << 32) | lo;
}
DEV u64 shfl64(u64 v, int src) {
  u32 lo = (u32)__shfl((int)(u32)v, src);
  u32 hi = (u32)__shfl((int)(u32)(v >> 32), src);
  return ((u64)hi << 32) | lo;
}
DEV u64 shfl_xor64(u64 v, int m) {
  u32 lo = (u32)__shfl_xor((int)(u32)v, m);
  u32 hi = (u32)__shfl_xor((int)(u32)(v >> 32), m);
  return ((u64)hi << 32) | lo;
}
DEV u64 shfl_up64(u64 v, int d) {
  u32 lo = (u32)__shfl_up((int)(u32)v, d);
  u32 hi = (u32)__shfl_up((int)(u32)(v >> 32), d);
  return ((u64)hi << 32) | lo;
}
DEV u64 wave_sum64(u64 v) {
  for (int m = 32; m > 0; m >>= 1) v += shfl_xor64(v, m);
  return v;
}

// ---- wave-distributed big integers ----------------------------------------
// Lane l holds 64-bit word l of a 4096-bit two's complement integer.  Sums of
// energies live in "X units" of 2^-1075, needing at most ~2150 bits, so the
// top lanes are sign extension.  Carries/borrows resolve in O(1) wave steps:
// with G = lanes that generate and P = lanes that propagate, the carry into
// every lane is ((G + (G|P)) ^ G ^ (G|P)).
DEV u64 carry_in(u64 G, u64 P) {
  u64 Y = G | P;
  return (G + Y) ^ G ^ Y;
}
DEV void wb_add(u64& w, u64 part) {
  u64 s = w + part;
  u64 c = carry_in(ballot(s < w), ballot(s == ~0ull));
  w = s + ((c >> lane_id()) & 1ull);
}
DEV void wb_sub(u64& w, u64 part) {
  u64 d = w - part;
  u64 c = carry_in(ballot(w < part), ballot(d == 0ull));
  w = d - ((c >> lane_id()) & 1ull);
}
// This lane's share of the 128-bit value (lo, hi) shifted left by s bits.
DEV u64 part_at(u64 lo, u64 hi, int s) {
  int q = s >> 6, r = s & 63, l = lane_id();
  if (l == q) return lo << r;
  if (l == q + 1) return r ? ((lo >> (64 - r)) | (hi << r)) : hi;
  if (l == q + 2) return r ? (hi >> (64 - r)) : 0ull;
  return 0ull;
}
DEV bool wb_neg(u64 w) { return (bcast64(w, 63) >> 63) != 0; }

// Round a non-negative big integer in X units to the nearest double (ties to
// even).
DEV double wb_round(u64 w) {
  u64 nz = ballot(w != 0);
  if (!nz) return 0.0;
  int L = 63 - __clzll((long long)nz);
  u64 top = bcast64(w, L);
  int t = 64 * L + 63 - __clzll((long long)top);  // highest set bit
  int lsb = t - 52 > 1 ? t - 52 : 1;              // X-unit weight of the result's ulp
  int q = lsb >> 6, r = lsb & 63;
  u64 a = bcast64(w, q);
  u64 b = (q + 1 < 64) ? bcast64(w, q + 1) : 0ull;
  u64 m = r ? ((a >> r) | (b << (64 - r))) : a;   // at most 53 significant bits
  int rb_pos = lsb - 1;
  int rq = rb_pos >> 6, rr = rb_pos & 63;
  u64 rw = bcast64(w, rq);
  u64 rbit = (rw >> rr) & 1ull;
  bool sticky = ((rw & ((1ull << rr) - 1ull)) != 0ull) || (ballot(w != 0 && lane_id() < rq) != 0ull);
  if (rbit && (sticky || (m & 1ull))) m += 1ull;
  return ldexp((double)m, lsb - 1075);
}

// 128 bits of the big integer starting at bit s; sat = bits above them exist.
DEV void wb_extract128(u64 w, int s, u64& lo, u64& hi, bool& sat) {
  int q = s >> 6, r = s & 63;
  u64 a = bcast64(w, q), b = bcast64(w, q + 1), c = bcast64(w, q + 2);
  lo = r ? ((a >> r) | (b << (64 - r))) : a;
  hi = r ? ((b >> r) | (c << (64 - r))) : b;
  u64 rest = r ? (c >> r) : c;
  sat = rest != 0ull || ballot(w != 0 && lane_id() > q + 2) != 0ull;
}

// Significand sum of one exponent bin as a 128-bit integer.
DEV u128 bin_sum(const HistBin& h) { return ((u128)h.hi << 21) + (u128)h.lo; }

// Lane l's exact sum of exponent bins [32 l, 32 l + 32), relative to
// X-unit shift base = max(32 l, 1); bin 2047 (non-finite) is excluded.
DEV void chunk32(const HistBin* H, u64& lo, u64& hi, u64& cnt, int& base) {
  int l = lane_id();
  base = 32 * l > 1 ? 32 * l : 1;
  u128 acc = 0;
  u64 c = 0;
  // all 32 bins are loaded before any is used (independent loads in flight)
  HistBin hb[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int b = 32 * l + k;
    hb[k] = b < HBINS - 1 ? H[b] : HistBin{0ull, 0ull, 0ull};
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int b = 32 * l + k;
    if (hb[k].cnt == 0) continue;
    int sh = (b > 1 ? b : 1) - base;
    acc += bin_sum(hb[k]) << sh;
    c += hb[k].cnt;
  }
  lo = (u64)acc;
  hi = (u64)(acc >> 64);
  cnt = c;
}

// Exact total of a histogram as a wave-distributed big integer.
DEV u64 hist_total(const HistBin* H) {
  u64 lo, hi, cnt;
  int base;
  chunk32(H, lo, hi, cnt, base);
  u64 acc = 0;
  for (int l = 0; l < 64; ++l) {
    u64 cl = bcast64(lo, l), ch = bcast64(hi, l);
    if ((cl | ch) == 0ull) continue;
    wb_add(acc, part_at(cl, ch, l == 0 ? 1 : 32 * l));
  }
  return acc;
}

// ---- LDS histogram window of one workgroup ----------------------------------
// HC copies of every bin (lane parity picks the copy) halve same-address
// atomic conflicts inside a wave.
constexpr int HC = 2;
struct LdsHist {
  u64 w[WIN][HC][2];  // [0] = (count << 43) + sum(sig & (2^21-1)), [1] = sum(sig >> 21)
  u32 zero;           // exact zeros
  int lo;             // exponent of w[0]
  int maxE;
  int pad;
};

DEV void lh_init(LdsHist& h, int tid, int nthr) {
  u64* p = &h.w[0][0][0];
  for (int k = tid; k < WIN * HC * 2; k += nthr) p[k] = 0ull;
  if (tid == 0) {
    h.zero = 0u;
    h.maxE = 0;
    h.lo = 0;
  }
}

DEV void global_bin_add(HistBin* g, int E, u64 cnt, u64 lo, u64 hi) {
  if (cnt) atomicAdd(&g[E].cnt, cnt);
  if (lo) atomicAdd(&g[E].lo, lo);
  if (hi) atomicAdd(&g[E].hi, hi);
}

DEV int bits_exp(u64 bits) {
  return (bits >> 63) ? 2047 : (int)(bits >> 52);  // negative = only NaN here
}

DEV void lh_insert(LdsHist& h, HistBin* g, double v) {
  u64 bits = dbits(v);
  if (bits == 0ull) {
    atomicAdd(&h.zero, 1u);
    return;
  }
  int E = bits_exp(bits);
  u64 sig = (bits & M52) | (E ? (1ull << 52) : 0ull);
  if (E == 2047) sig = 0;
  int b = E - h.lo;
  if ((unsigned)b < (unsigned)WIN) {
    const int cp = lane_id() & (HC - 1);
    atomicAdd(&h.w[b][cp][0], (1ull << 43) + (sig & M21));
    atomicAdd(&h.w[b][cp][1], sig >> 21);
  } else {
    global_bin_add(g, E, 1ull, sig & M21, sig >> 21);
  }
}

// Window placement from the largest exponent seen in the first tile.
DEV void lh_note_max(LdsHist& h, double v) {
  int E = bits_exp(dbits(v));
  if (E > 0 && E < 2047) atomicMax(&h.maxE, E);
}
DEV void lh_place(LdsHist& h) { h.lo = h.maxE + WIN_HEAD - WIN + 1; }

DEV void lh_flush(LdsHist& h, HistBin* g, int tid, int nthr) {
  for (int b = tid; b < WIN; b += nthr) {
    u64 cnt = 0, lo = 0, hi = 0;
    for (int cp = 0; cp < HC; ++cp) {
      const u64 w0 = h.w[b][cp][0];
      cnt += w0 >> 43;
      lo += w0 & M43;
      hi += h.w[b][cp][1];
    }
    if (cnt | lo | hi) global_bin_add(g, h.lo + b, cnt, lo, hi);
  }
  if (tid == 0 && h.zero) atomicAdd(&g[0].cnt, (u64)h.zero);
}

// ---- candidate lists -------------------------------------------------------------
// Per component: list 0 (capacity list_cap) then lists 1 and 2 (list_cap / 2
// each; they only hold the members of one refinement sub-bin).
DEV u64* list_ptr(const Job& j, int comp, int k) {
  return j.lists + (size_t)comp * 2 * j.list_cap + (k == 0 ? 0 : j.list_cap + (size_t)(k - 1) * (j.list_cap / 2));
}
DEV u64 list_capk(const Job& j, int k) { return k == 0 ? j.list_cap : j.list_cap / 2; }

// Wave-aggregated append; the counter may run past cap (then ST_LIST is set
// and readers clamp to cap).
DEV void list_append(u64* list, u64* count, u64 cap, bool m, u64 key, int* flag) {
  const u64 bal = ballot(m);
  if (bal == 0ull) return;
  const int leader = __ffsll((long long)bal) - 1;
  u64 base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (u64)__popcll(bal));
  base = shfl64(base, leader);
  if (m) {
    const u64 pos = base + (u64)__popcll(bal & ((1ull << lane_id()) - 1ull));
    if (pos < cap)
      list[pos] = key;
    else
      atomicOr(flag, ST_LIST);
  }
}

// ---- decoupled look-back --------------------------------------------------------
// Descriptor per tile: flag << 62 | value; flag 1 = aggregate, 2 = inclusive
// prefix.  publish() posts the tile's aggregate (tile 0 posts its prefix);
// wait() reads 64 predecessors at a time (lane i: tile base - i) until one
// carries an inclusive prefix, then posts the tile's own prefix.  Both run on
// one whole wave.
DEV u64 lb_load(const u64* p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT); }
DEV void lb_store(u64* p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }

DEV u64 tile_agg(const u32* cntl, int ne) {
  u64 agg = 0;
  for (int k = 0; k < ne; ++k) agg += cntl[k];
  return agg;
}

DEV void lookback_publish(u64* lb, long long t, const u32* cntl, int ne, u64* excl_out) {
  if (lane_id() != 0) return;
  const u64 agg = tile_agg(cntl, ne);
  if (t == 0) {
    lb_store(&lb[0], (2ull << 62) | agg);
    *excl_out = 0ull;
  } else {
    lb_store(&lb[t], (1ull << 62) | agg);
  }
}

constexpr int SPIN_LIMIT = 1 << 24;

DEV void lookback_wait(u64* lb, long long t, const u32* cntl, int ne, int* flags, u64* excl_out) {
  if (t == 0) return;
  const int lane = lane_id();
  u64 ex = 0;
  long long base = t - 1;
  for (;;) {
    const long long idx = base - lane;
    u64 sv = 2ull << 62;  // before tile 0: an inclusive prefix of 0
    if (idx >= 0) {
      int spins = 0;
      for (;;) {
        sv = lb_load(&lb[idx]);
        if ((sv >> 62) != 0ull || ++spins >= SPIN_LIMIT) break;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (ballot((sv >> 62) == 0ull)) {  // a predecessor never published (cannot happen)
      if (lane == 0) atomicOr(flags, ST_SPIN);
      break;
    }
    const u64 pm = ballot((sv >> 62) == 2ull);
    const int stop = pm ? (__ffsll((long long)pm) - 1) : 63;
    ex += wave_sum64(lane <= stop ? (sv & M62) : 0ull);
    if (pm) break;
    base -= 64;
  }
  if (lane == 0) {
    lb_store(&lb[t], (2ull << 62) | (ex + tile_agg(cntl, ne)));
    *excl_out = ex;
  }
}

// ---- FP64 fixed-order contraction ---------------------------------------------
// y[a] = M[a][0]*x[0] + M[a][1]*x[1] + ... left to right, every product and
// sum rounded separately (the library is built with -ffp-contract=off).
template <int n>
DEV void contract64(const double* __restrict__ M, const double (&x)[n], double (&y)[n]) {
#pragma unroll
  for (int a = 0; a < n; ++a) {
    // keep the row loads of M here (LDS broadcast reads) instead of letting
    // the compiler hold all n*n entries in VGPRs across stages
    asm volatile("" ::: "memory");
    double acc = M[a * n] * x[0];
#pragma unroll
    for (int b = 1; b < n; ++b) acc = acc + M[a * n + b] * x[b];
    y[a] = acc;
  }
}

// Coalesced copy of `count` doubles from global to LDS.
template <int THREADS>
DEV void load_tile(double* __restrict__ dst, const double* __restrict__ src, int count, int tid) {
  if ((((uintptr_t)src) & 15) == 0 && (count & 1) == 0) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
    double2* d2 = reinterpret_cast<double2*>(dst);
    for (int k = tid; k < (count >> 1); k += THREADS) d2[k] = s2[k];
  } else {
    for (int k = tid; k < count; k += THREADS) dst[k] = src[k];
  }
}


}  // namespace isr
