// Streaming path for orders 1..7 ((N+1)^2 <= 64): one wavefront owns a tile
// of EPW = 64 / (N+1)^2 elements and runs its whole transform chain on its
// own, with no workgroup barriers.
//
//   k_sample  every sample_stride-th tile: rounded exponent histogram of the
//             energies and rounded U2, which place a window of three energy
//             exponent bins around the expected threshold
//   k_passA   exact norm sum, sum of the energies below the window, window
//             energies (with their element) to list 0, per-element count of
//             energies above the window
//   k_passB   keep e >= tau, bitmaps, kept values at per-element offsets
//             (known up front: no look-back), inverse of the kept set, error
//             sum; the last workgroup of a component finalizes it
//
// Exact sums without atomics: every lane splits each non-negative term x <= M
// into three parts on fixed grids (error-free extraction against fixed powers
// of two, Rump, Ogita and Oishi, "Accurate floating-point summation part I",
// SIAM J. Sci. Comput. 31(1), 2008, Alg. 3.2) and keeps three FP64 running
// sums that stay exact; the rare term that leaves a remainder (far below M or
// above M) goes to the global exponent bins instead.  Workgroups publish
// their three integer sums; the consumer turns the totals into exact bins.
// The norm sum is exact on every path, so U2 is that of the FP64 field.  The
// FP64 path sums the energies and the error terms the same way; the MFMA
// paths, whose energies already carry the transform error, add them in a
// fixed order per lane instead (one FP64 add a term) and split only each
// lane's total on the grids, so their results stay deterministic.
//
// Transforms on MFMA use a block-diagonal trick for n <= 8: a 16x16 tile
// holds two 8x8 copies of the 1D matrix, the K dimension pairs the contracted
// index of two sets of 16 pencils, so the 64 lanes of every output register
// hold 64 valid (pencil, index) pairs.  Lane l = 16 g + P of block b holds
// pencil 32 b + 16 (g >> 1) + P and indices 4 (g & 1) + m, m = 0..3, in
// four registers, for the input and for the output of every stage alike.
// Between stages the tile is transposed through a per-wave LDS buffer.
// The FP64 path keeps one pencil per lane and the fixed evaluation order of
// the oracle (contract64).
#pragma once

#include "isr_passes.cuh"
#include "isr_fastsel.cuh"
#include "isr_selbody.cuh"
#include "isr_xsum.cuh"

// Minimum resident workgroups per CU the streaming passes are compiled for
// (bounds their registers: 4 -> 128 VGPRs, 3 -> 168, 2 -> 256).  Measured on
// the 65,536-element N = 7 snapshot: the FP64 transforms want 2 (fewer
// workgroups beat spilling), the MFMA paths 3.
#ifndef ISR_FAST_MINB_F64
#define ISR_FAST_MINB_F64 2
#endif
#ifndef ISR_FAST_MINB_MIX
#define ISR_FAST_MINB_MIX 3
#endif
#define ISR_FAST_MINB (PREC == P_FP64 ? ISR_FAST_MINB_F64 : ISR_FAST_MINB_MIX)

namespace isr {

template <bool C, class A, class B>
struct Pick {
  typedef A type;
};
template <class A, class B>
struct Pick<false, A, B> {
  typedef B type;
};

// ---- the wave-tile engine --------------------------------------------------------
template <int N, int PREC>
struct Eng {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static_assert(n >= 2 && n <= 8, "streaming engine covers orders 1..7");
  static constexpr bool MF = PREC != P_FP64;
  static constexpr int EPW = 64 / n2;      // elements per tile
  static constexpr int PT = EPW * n2;      // pencils per tile (<= 64)
  static constexpr int NB = MF ? 2 : 1;    // pencil blocks (32 pencils each on MFMA)
  static constexpr int SPB = MF ? 4 : n;   // registers per block
  static constexpr int NS = NB * SPB;      // slots per lane
  static_assert(NS <= 8, "slot tables hold 8 slots");
  static constexpr int P0 = n + 1;         // LDS row pitch
  static constexpr int LDSW = EPW * n * n * P0;
  static constexpr int W = (n3 + 63) / 64;  // bitmap words per element
  typedef typename Pick<MF, float, double>::type wt;

  struct Mats {
    float fa[4], fv[4];  // FP32 A-operand fragments (forward A, inverse V)
    s4 ha, la, hv, lv;   // BF16 hi / lo fragments
  };

  DEV static int pencil(int s, int lane) { return MF ? 32 * (s >> 2) + 16 * (lane >> 5) + (lane & 15) : lane; }
  DEV static int axis(int s, int lane) { return MF ? 4 * ((lane >> 4) & 1) + (s & 3) : s; }
  DEV static bool pvalid(int s, int lane) { return pencil(s, lane) < PT && axis(s, lane) < n; }
  DEV static bool valid(int s, int lane, int ne) { return pencil(s, lane) < ne * n2 && axis(s, lane) < n; }
  DEV static int elem(int s, int lane) { return pencil(s, lane) / n2; }

  static DEV void frag(float (&f)[4], s4& h, s4& l, const float* M, int lane) {
    const int row = lane & 15, g = lane >> 4;
    const bool same = (row >> 3) == (g >> 1);
    const int b = row & 7;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 4 * (g & 1) + v;
      const float m = (same && b < n && a < n) ? M[b * n + a] : 0.0f;
      f[v] = m;
      const short hi = to_bf16(m);
      h[v] = hi;
      l[v] = to_bf16(m - from_bf16(hi));
    }
  }
  static DEV void init(Mats& mt, const DevTables& t, int lane) {
    if constexpr (MF) {
      frag(mt.fa, mt.ha, mt.la, t.A32, lane);
      frag(mt.fv, mt.hv, mt.lv, t.V32, lane);
    }
  }

  // FP64 field tile -> slots (zero outside the tile).
  static DEV void load(const double* __restrict__ tile, int ne, bool vec, double (&u)[NS], int lane) {
    const int pv = ne * n2;
    if (n == 8 && vec) {
#pragma unroll
      for (int blk = 0; blk < NB; ++blk) {
        const int PI = pencil(blk * SPB, lane);
        const int a0 = axis(blk * SPB, lane);
#pragma unroll
        for (int h = 0; h < SPB / 2; ++h) {
          d2 v = {0.0, 0.0};
          if (PI < pv) v = __builtin_nontemporal_load((const d2*)(tile + PI * n + a0 + 2 * h));
          u[blk * SPB + 2 * h] = v.x;
          u[blk * SPB + 2 * h + 1] = v.y;
        }
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int PI = pencil(s, lane), ax = axis(s, lane);
      u[s] = (PI < pv && ax < n) ? __builtin_nontemporal_load(tile + PI * n + ax) : 0.0;
    }
  }

  // One contraction on every pencil of the tile.
  static DEV void stage_mf(const wt (&x)[NS], wt (&y)[NS], const float (&f)[4], s4 h, s4 l) {
    static_assert(MF, "MFMA stage");
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      f4 d = {0.0f, 0.0f, 0.0f, 0.0f};
      if (PREC == P_FP32) {
#pragma unroll
        for (int s = 0; s < 4; ++s) d = __builtin_amdgcn_mfma_f32_16x16x4f32(f[s], (float)x[4 * blk + s], d, 0, 0, 0);
      } else {
        s4 xh, xl;
        split_bf16x4((float)x[4 * blk], (float)x[4 * blk + 1], (float)x[4 * blk + 2], (float)x[4 * blk + 3], xh, xl);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, xh, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(l, xh, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, xl, d, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) y[4 * blk + v] = (wt)d[v];
    }
  }

  // LDS coordinates (e, x2, x1, x0) of a (pencil, index) pair; the pencil's
  // own two coordinates are (a, b) = ((PI % n2) / n, PI % n).
  //   pattern 1: (a, b, ax)   pattern 2: (a, ax, b)   pattern 3: (ax, a, b)
  template <int PAT>
  static DEV int addr(int PI, int ax) {
    const int e = PI / n2, rem = PI % n2, a = rem / n, b = rem % n;
    const int x2 = PAT == 3 ? ax : a;
    const int x1 = PAT == 1 ? b : (PAT == 2 ? ax : a);
    const int x0 = PAT == 1 ? ax : b;
    return ((e * n + x2) * n + x1) * P0 + x0;
  }
  // n = 8 (one element per tile, every slot valid): the address is a lane
  // part plus a per-slot constant, so that every access is one base register
  // with an immediate offset.
  template <int PAT>
  static DEV int lane_part(int lane) {
    if constexpr (MF) {
      const int P = lane & 15, hs = lane >> 5, gl = (lane >> 4) & 1;
      const int a = 2 * hs + (P >> 3), b = P & 7;
      if constexpr (PAT == 1) return (a * 8 + b) * P0 + 4 * gl;
      if constexpr (PAT == 2) return (a * 8 + 4 * gl) * P0 + b;
      return (32 * gl + a) * P0 + b;
    } else {
      const int a = lane >> 3, b = lane & 7;
      if constexpr (PAT == 1) return (a * 8 + b) * P0;
      if constexpr (PAT == 2) return a * 8 * P0 + b;
      return a * P0 + b;
    }
  }
  template <int PAT>
  static constexpr int slot_part(int s) {
    if constexpr (MF) {
      const int blk = s >> 2, m = s & 3;
      if constexpr (PAT == 1) return 32 * P0 * blk + m;
      if constexpr (PAT == 2) return 32 * P0 * blk + m * P0;
      return (8 * m + 4 * blk) * P0;
    } else {
      if constexpr (PAT == 1) return s;
      if constexpr (PAT == 2) return s * P0;
      return 8 * s * P0;
    }
  }
  template <int WP, int RP>
  static DEV void xpose(const wt (&y)[NS], wt (&x)[NS], wt* buf, int lane) {
    if constexpr (n == 8) {
      wt* bw = buf + lane_part<WP>(lane);
      const wt* br = buf + lane_part<RP>(lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) bw[slot_part<WP>(s)] = y[s];
      asm volatile("" ::: "memory");
#pragma unroll
      for (int s = 0; s < NS; ++s) x[s] = br[slot_part<RP>(s)];
      asm volatile("" ::: "memory");
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (pvalid(s, lane)) buf[addr<WP>(pencil(s, lane), axis(s, lane))] = y[s];
      asm volatile("" ::: "memory");
#pragma unroll
      for (int s = 0; s < NS; ++s) x[s] = pvalid(s, lane) ? buf[addr<RP>(pencil(s, lane), axis(s, lane))] : (wt)0;
      asm volatile("" ::: "memory");
    }
  }

  // forward: contract i (pattern 1 -> 2), j (2 -> 3), k; slots of the field
  // tile in, slots of the coefficients (pencil (q, p), index r) out
  static DEV void forward(const double (&u)[NS], double (&c)[NS], wt* buf, const Mats& mt, const DevTables& t,
                          int lane) {
    wt x[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = (wt)u[s];
    if constexpr (MF) {
      stage_mf(x, y, mt.fa, mt.ha, mt.la);
      xpose<1, 2>(y, x, buf, lane);
      stage_mf(x, y, mt.fa, mt.ha, mt.la);
      xpose<2, 3>(y, x, buf, lane);
      stage_mf(x, y, mt.fa, mt.ha, mt.la);
    } else {
      contract64<n>(t.A, x, y);
      xpose<1, 2>(y, x, buf, lane);
      contract64<n>(t.A, x, y);
      xpose<2, 3>(y, x, buf, lane);
      contract64<n>(t.A, x, y);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) c[s] = (double)y[s];
  }

  // inverse: contract r (3 -> 2), q (2 -> 1), p; coefficient slots in, field
  // slots out
  static DEV void inverse(const double (&cm)[NS], double (&ut)[NS], wt* buf, const Mats& mt, const DevTables& t,
                          int lane) {
    wt x[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = (wt)cm[s];
    if constexpr (MF) {
      stage_mf(x, y, mt.fv, mt.hv, mt.lv);
      xpose<3, 2>(y, x, buf, lane);
      stage_mf(x, y, mt.fv, mt.hv, mt.lv);
      xpose<2, 1>(y, x, buf, lane);
      stage_mf(x, y, mt.fv, mt.hv, mt.lv);
    } else {
      contract64<n>(t.V, x, y);
      xpose<3, 2>(y, x, buf, lane);
      contract64<n>(t.V, x, y);
      xpose<2, 1>(y, x, buf, lane);
      contract64<n>(t.V, x, y);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) ut[s] = (double)y[s];
  }

  // Table indices of the slots: w3 for field slots, g3 for coefficient slots
  // (n = 8: a lane part plus a per-slot constant).
  DEV static int w3i(int s, int lane) {
    if constexpr (n == 8 && MF) return ((lane >> 5) * 16 + (lane & 15)) * 8 + 4 * ((lane >> 4) & 1) + (256 * (s >> 2) + (s & 3));
    if constexpr (n == 8) return lane * 8 + s;
    return (pencil(s, lane) % n2) * n + axis(s, lane);
  }
  DEV static int g3i(int s, int lane) {
    if constexpr (n == 8 && MF) return (256 * ((lane >> 4) & 1) + (lane >> 5) * 16 + (lane & 15)) + (64 * (s & 3) + 32 * (s >> 2));
    if constexpr (n == 8) return s * 64 + lane;
    return axis(s, lane) * n2 + pencil(s, lane) % n2;
  }

  // OR the kept bits of slot s (ballot m) into the tile's bitmap words in LDS
  // (bm[ee * W + w]); wave-uniform, one lane writes.
  static DEV void bitmap_or(u64* bm, u64 m, int s, int ne, int lane) {
    constexpr int RUNS = MF ? 4 : 1, RLEN = MF ? 16 : 64;
#pragma unroll
    for (int g = 0; g < RUNS; ++g) {
      const int L0 = g * RLEN;
      const int PI0 = pencil(s, L0), ax = axis(s, L0);
      if (ax >= n) continue;
      const u64 bits = RLEN == 64 ? m : ((m >> L0) & ((1ull << RLEN) - 1ull));
      int pos = 0;
      while (pos < RLEN && (bits >> pos) != 0ull) {
        const int PI = PI0 + pos;
        const int ee = PI / n2;
        if (ee >= ne) break;
        const int rem = PI % n2;
        const int c = (RLEN - pos) < (n2 - rem) ? (RLEN - pos) : (n2 - rem);
        const u64 chunk = (bits >> pos) & (c >= 64 ? ~0ull : ((1ull << c) - 1ull));
        if (chunk && lane == 0) {
          const int f0 = ax * n2 + rem, w = f0 >> 6, o = f0 & 63;
          atomicOr(&bm[ee * W + w], chunk << o);
          if (o && o + c > 64) atomicOr(&bm[ee * W + w + 1], chunk >> (64 - o));
        }
        pos += c;
      }
    }
  }
};

// w3 and g3 of every (slot, lane) in LDS, slot-major so that the 64 lanes of
// a read hit 64 consecutive doubles (registers would cost 4 NS VGPRs).
struct TabLds {
  double w3[8][64], g3[8][64];
};
template <class G>
DEV void tab_load(TabLds& T, const DevTables& t, int tid) {
  for (int k = tid; k < G::NS * 64; k += 256) {
    const int s = k >> 6, l = k & 63;
    const bool v = G::pvalid(s, l);
    T.w3[s][l] = v ? t.w3[G::w3i(s, l)] : 0.0;
    T.g3[s][l] = v ? t.g3[G::g3i(s, l)] : 0.0;
  }
}

// ---- sample pass --------------------------------------------------------------
constexpr int SBINS = HBINS;

template <int N, int PREC>
struct SampleLds {
  typename Eng<N, PREC>::wt buf[4][Eng<N, PREC>::LDSW];
  TabLds tab;
  u32 hc[SBINS];
  float hs[SBINS];  // sums of energy / 2^(bin exponent), each term in [1, 2)
  double u2[4];
  int maxe;
  int last;
};

template <int N, int PREC>
DEV void sample_body(const Job& j, int comp, int vb, int nvb, SampleLds<N, PREC>& L, bool tail) {
  typedef Eng<N, PREC> G;
  constexpr int n3 = G::n3, NS = G::NS, EPW = G::EPW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  for (int k = tid; k < SBINS; k += 256) {
    L.hc[k] = 0u;
    L.hs[k] = 0.0f;
  }
  if (tid == 0) L.maxe = 0;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tab_load<G>(L.tab, j.tab, tid);
  __syncthreads();
  __syncthreads();
  const long long E = j.n_elem, tiles = (E + EPW - 1) / EPW;
  const long long ss = j.sample_stride > 0 ? j.sample_stride : 1;
  const long long stiles = (tiles + ss - 1) / ss;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const bool vec = ((((uintptr_t)ub) & 15) == 0);
  const long long nw = (long long)nvb * 4;
  double u2 = 0.0;
  int maxe = 0;
  for (long long k = (long long)vb * 4 + wv; k < stiles; k += nw) {
    const long long t = k * ss;
    const long long e0 = t * EPW;
    const int ne = (int)((E - e0) < EPW ? (E - e0) : EPW);
    double u[NS], c[NS];
    G::load(ub + e0 * n3, ne, vec, u, lane);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!G::valid(s, lane, ne)) continue;
      const double x = jw(j.jac, e0 + G::elem(s, lane), L.tab.w3[s][lane]) * (u[s] * u[s]);
      u2 += x;
      const int ex = bits_exp(dbits(x));
      maxe = ex > maxe ? ex : maxe;
    }
    G::forward(u, c, L.buf[wv], mt, j.tab, lane);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const bool v = G::valid(s, lane, ne);
      const double en = v ? jw(j.jac, e0 + G::elem(s, lane), L.tab.g3[s][lane]) * (c[s] * c[s]) : 0.0;
      const int b = bits_exp(dbits(en));
      if (v && b < HBINS - 1) {  // rounded sums only place the window
        atomicAdd(&L.hc[b], 1u);
        atomicAdd(&L.hs[b], (float)ldexp(en, 1023 - b));
      }
    }
  }
  u2 = wave_sum_f64(u2);
  for (int m = 32; m > 0; m >>= 1) {
    const int o = __shfl_xor(maxe, m);
    maxe = o > maxe ? o : maxe;
  }
  if (lane == 0) {
    L.u2[wv] = u2;
    atomicMax(&L.maxe, maxe);
  }
  __syncthreads();
  HistBin* H = j.histEs + (size_t)comp * HBINS;
  for (int k = tid; k < SBINS; k += 256) {
    if (L.hc[k]) {
      atomicAdd((double*)&H[k].lo, ldexp((double)L.hs[k], k - 1023));
    }
  }
  if (tid == 0) {
    atomicAdd(&st->samp_u2, L.u2[0] + L.u2[1] + L.u2[2] + L.u2[3]);
    atomicMax(&st->samp_maxe, L.maxe);
  }
  if (!tail || !last_block(j.done + D_SAMPLE * 8 + comp, &L.last, nvb)) return;
  if (tid < 64) select_sample_body(j, comp);
}

template <int N, int PREC>
__global__ __launch_bounds__(256, ISR_FAST_MINB) void k_sample(Job j) {
  __shared__ SampleLds<N, PREC> L;
  sample_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

// ---- pass A -------------------------------------------------------------------
constexpr int CAPB = 256;  // per-wave staging of window candidates

template <int N, int PREC>
struct PassALds {
  typename Eng<N, PREC>::wt buf[4][Eng<N, PREC>::LDSW];
  TabLds tab;
  u64 key[4][CAPB];
  u32 idx[4][CAPB];
  u32 ecnt[4][16];
  long long red[4][8];
};

DEV void cap_flush(u64* key, u32* idx, u32& ncap, CompState* st, u64* list, u32* lidx, u64 cap, int lane) {
  if (ncap == 0u) return;
  u64 base = 0ull;
  if (lane == 0) base = atomicAdd(&st->list_count[0], (u64)ncap);
  base = bcast64(base, 0);
  for (u32 i = lane; i < ncap; i += 64) {
    const u64 pos = base + i;
    if (pos < cap) {
      list[pos] = key[i];
      lidx[pos] = idx[i];
    } else {
      atomicOr(&st->flags, ST_LIST);
    }
  }
  ncap = 0u;
  asm volatile("" ::: "memory");
}

template <int N, int PREC>
DEV void passA_body(const Job& j, int comp, int vb, int nvb, PassALds<N, PREC>& L) {
  typedef Eng<N, PREC> G;
  constexpr int n3 = G::n3, NS = G::NS, EPW = G::EPW;
  constexpr bool EXACT = PREC == P_FP64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const int wlo = st->win_lo, whi = st->win_hi;
  const XParm PN = xparm(st->xm_norm, j.xh);
  const XParm PE = xparm(wlo - 1023, j.xh);
  HistBin* gN = j.histN + (size_t)comp * HBINS;
  HistBin* gE = j.histE + (size_t)comp * HBINS;
  u64* list = list_ptr(j, comp, 0);
  u32* lidx = j.lidx + (size_t)comp * j.list_cap;
  const long long E = j.n_elem, tiles = (E + EPW - 1) / EPW;
  u32* cnt = j.cnt + (size_t)comp * E;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tab_load<G>(L.tab, j.tab, tid);
  __syncthreads();
  XAcc an = {0.0, 0.0, 0.0}, ae = {0.0, 0.0, 0.0};
  double pe = 0.0;  // fixed-order sum of the energies below the window
  double pn = 0.0;  // MFMA paths: fixed-order sum of the norm terms
  u64 hi_tot = 0ull;
  u32 ncap = 0u;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const bool vec = ((((uintptr_t)ub) & 15) == 0);
  const long long nw = (long long)nvb * 4;
  // the next tile's field values are loaded while this one is processed
  double un[NS];
  {
    const long long t0 = (long long)vb * 4 + wv;
    if (t0 < tiles) G::load(ub + t0 * EPW * n3, (int)((E - t0 * EPW) < EPW ? (E - t0 * EPW) : EPW), vec, un, lane);
  }
  for (long long t = (long long)vb * 4 + wv; t < tiles; t += nw) {
    const long long e0 = t * EPW;
    const int ne = (int)((E - e0) < EPW ? (E - e0) : EPW);
    double u[NS], c[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) u[s] = un[s];
    if (t + nw < tiles) {
      const long long e1 = (t + nw) * EPW;
      G::load(ub + e1 * n3, (int)((E - e1) < EPW ? (E - e1) : EPW), vec, un, lane);
    }
    // quadrature weights of the slots (times the element's Jacobian), with the
    // Jacobian test taken once per tile
    double wq[NS];
    if (j.jac) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        wq[s] = G::valid(s, lane, ne) ? j.jac[e0 + G::elem(s, lane)] * L.tab.w3[s][lane] : 0.0;
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) wq[s] = L.tab.w3[s][lane];
    }
    // norm terms: every term split exactly on the FP64 path; on the MFMA
    // paths each lane sums its terms in a fixed FP64 order and only the lane
    // totals are added exactly (as for the energies and the error terms)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double x = G::valid(s, lane, ne) ? wq[s] * (u[s] * u[s]) : 0.0;
      if constexpr (EXACT) {
        double r;
        if (xadd_left(an, PN, x, r)) slow_bin(gN, r);
        // one slot at a time: interleaving them would hold every slot's
        // temporaries at once and cut the occupancy
        __builtin_amdgcn_sched_barrier(0);
      } else {
        pn += x;
      }
    }
    G::forward(u, c, L.buf[wv], mt, j.tab, lane);
    if (EPW > 1) {
      if (lane < EPW) L.ecnt[wv][lane] = 0u;
      asm volatile("" ::: "memory");
    }
    u32 hc = 0u;
    if (j.jac) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        wq[s] = G::valid(s, lane, ne) ? j.jac[e0 + G::elem(s, lane)] * L.tab.g3[s][lane] : 0.0;
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) wq[s] = L.tab.g3[s][lane];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const bool v = G::valid(s, lane, ne);
      const double en = v ? wq[s] * (c[s] * c[s]) : 0.0;
      const u64 key = dbits(en);
      const int ex = bits_exp(key);
      const bool hi = v && ex >= whi;
      const bool cp = v && ex < whi && ex >= wlo;
      const bool nf = hi && ex == HBINS - 1;  // Inf/NaN: counted in the flag bin
      // the wave votes first: lane flags that stay live across the divergent
      // branches below would be copied through vector registers on every slot
      const u64 bh = ballot(hi);
      const u64 bc = ballot(cp);
      hc += (u32)__popcll(bh);
      if (EPW > 1 && hi) atomicAdd(&L.ecnt[wv][G::elem(s, lane)], 1u);
      if (bc) {
        const u32 pos = ncap + (u32)__popcll(bc & ((1ull << lane) - 1ull));
        if (cp) {
          L.key[wv][pos] = key;
          L.idx[wv][pos] = (u32)(e0 + G::elem(s, lane));
        }
        ncap += (u32)__popcll(bc);
        if (ncap > (u32)(CAPB - 64)) {
          asm volatile("" ::: "memory");
          cap_flush(L.key[wv], L.idx[wv], ncap, st, list, lidx, j.list_cap, lane);
        }
      }
      if constexpr (EXACT) {
        double r = xadd_r(ae, PE, (v && ex < wlo) ? en : 0.0);
        if (nf) r = en;
        if (r != 0.0) slow_bin(gE, r);
      } else {
        pe += (v && ex < wlo) ? en : 0.0;
        if (nf) slow_bin(gE, en);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    hi_tot += hc;
    if (EPW == 1) {
      if (lane == 0) cnt[e0] = hc;
    } else {
      asm volatile("" ::: "memory");
      if (lane < ne) cnt[e0 + lane] = L.ecnt[wv][lane];
    }
  }
  asm volatile("" ::: "memory");
  cap_flush(L.key[wv], L.idx[wv], ncap, st, list, lidx, j.list_cap, lane);
  if constexpr (!EXACT) {
    const double r = xadd_sum(ae, PE, pe);
    if (r != 0.0) slow_bin(gE, r);
    const double rn = xadd_sum(an, PN, pn);
    if (rn != 0.0) slow_bin(gN, rn);
  }
  long long v[7];
  long long kn[3], ke[3];
  xints(an, PN, kn);
  xints(ae, PE, ke);
  v[0] = kn[0];
  v[1] = kn[1];
  v[2] = kn[2];
  v[3] = ke[0];
  v[4] = ke[1];
  v[5] = ke[2];
  v[6] = lane == 0 ? (long long)hi_tot : 0ll;
  block_sum_i64<7>(v, L.red, tid);
  if (tid < 7) j.slotsA[((size_t)comp * j.gA + vb) * 8 + tid] = L.red[0][tid];
}

template <int N, int PREC>
__global__ __launch_bounds__(256, ISR_FAST_MINB) void k_passA(Job j) {
  __shared__ PassALds<N, PREC> L;
  passA_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L);
}

// ---- pass B -------------------------------------------------------------------
template <int N, int PREC>
struct PassBLds {
  typename Eng<N, PREC>::wt buf[4][Eng<N, PREC>::LDSW];
  TabLds tab;
  u64 bm[4][16];
  u32 wp[4][16];
  long long red[4][8];
  __int128 r3[4][3];
  int last;
};

template <int N, int PREC>
DEV void passB_body(const Job& j, int comp, int vb, int nvb, PassBLds<N, PREC>& L, bool tail) {
  typedef Eng<N, PREC> G;
  constexpr int n3 = G::n3, NS = G::NS, EPW = G::EPW, W = G::W;
  constexpr bool EXACT = PREC == P_FP64;
  static_assert(EPW * W <= 16, "tile bitmap fits the LDS slot");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const XParm PR = xparm(st->xm_err, j.xh);
  HistBin* gR = j.histR + (size_t)comp * HBINS;
  const u64 tk = dbits(st->tau);
  u64 voff = 0ull;
  for (int cc = 0; cc < comp; ++cc) voff += j.st[cc].kept;
  const u64 vcap = (u64)j.ncomp * (u64)j.n_elem * (u64)n3;
  const long long E = j.n_elem, tiles = (E + EPW - 1) / EPW;
  const u64* eptr = j.elem_ptr + (size_t)comp * (E + 1);
  u64* gbm = j.bitmap + (size_t)comp * E * W;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tab_load<G>(L.tab, j.tab, tid);
  __syncthreads();
  XAcc ar = {0.0, 0.0, 0.0};
  double pr = 0.0;  // fixed-order sum of the error terms
  bool bad = false;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const bool vec = ((((uintptr_t)ub) & 15) == 0);
  const long long nw = (long long)nvb * 4;
  u64* bm = L.bm[wv];
  u32* wp = L.wp[wv];
  // the next tile's field values are loaded while this one is processed
  double un[NS];
  {
    const long long t0 = (long long)vb * 4 + wv;
    if (t0 < tiles) G::load(ub + t0 * EPW * n3, (int)((E - t0 * EPW) < EPW ? (E - t0 * EPW) : EPW), vec, un, lane);
  }
  for (long long t = (long long)vb * 4 + wv; t < tiles; t += nw) {
    const long long e0 = t * EPW;
    const int ne = (int)((E - e0) < EPW ? (E - e0) : EPW);
    double u[NS], c[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) u[s] = un[s];
    if (t + nw < tiles) {
      const long long e1 = (t + nw) * EPW;
      G::load(ub + e1 * n3, (int)((E - e1) < EPW ? (E - e1) : EPW), vec, un, lane);
    }
    G::forward(u, c, L.buf[wv], mt, j.tab, lane);
    // energy weights of the slots (times the element's Jacobian), with the
    // Jacobian test taken once per tile
    double wq[NS];
    if (j.jac) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        wq[s] = G::valid(s, lane, ne) ? j.jac[e0 + G::elem(s, lane)] * L.tab.g3[s][lane] : 0.0;
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) wq[s] = L.tab.g3[s][lane];
    }
    bool keep[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const bool v = G::valid(s, lane, ne);
      const double en = v ? wq[s] * (c[s] * c[s]) : 0.0;
      keep[s] = v && dbits(en) >= tk;
    }
    if constexpr (G::n == 8) {
      // one element per tile and one 64-bit word per index r: the words come
      // straight from the ballots (wave-uniform, no LDS)
      u64 B[NS], word[8];
#pragma unroll
      for (int s = 0; s < NS; ++s) B[s] = ballot(keep[s]);
      if constexpr (G::MF) {
        // slot s = 4 blk + m on lane 16 g + P: index r = 4 (g & 1) + m, pencil
        // 32 blk + 16 (g >> 1) + P
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = r & 3, gl = r >> 2;
          u64 w = 0ull;
#pragma unroll
          for (int blk = 0; blk < 2; ++blk)
#pragma unroll
            for (int hs = 0; hs < 2; ++hs)
              w |= ((B[4 * blk + m] >> (16 * (2 * hs + gl))) & 0xFFFFull) << (32 * blk + 16 * hs);
          word[r] = w;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) word[r] = B[r];
      }
      u32 pre[8];
      u32 tot = 0u;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        pre[r] = tot;
        tot += (u32)__popcll(word[r]);
      }
      u64 mine = 0ull;
#pragma unroll
      for (int r = 0; r < 8; ++r) mine = lane == r ? word[r] : mine;
      // bits below this lane's pencil in its words (one mask per pencil block)
      u64 below[G::NB];
#pragma unroll
      for (int blk = 0; blk < G::NB; ++blk) below[blk] = (1ull << G::pencil(blk * G::SPB, lane)) - 1ull;
      if (lane < 8) gbm[e0 * 8 + lane] = mine;
      const u64 ebase = eptr[e0];
      if ((u64)tot != eptr[e0 + 1] - ebase) bad = true;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (!keep[s]) continue;
        u64 wd;
        u32 pr;
        if constexpr (G::MF) {  // index r = 4 (g & 1) + (s & 3): one of two words
          const bool up = (lane >> 4) & 1;
          wd = up ? word[4 + (s & 3)] : word[s & 3];
          pr = up ? pre[4 + (s & 3)] : pre[s & 3];
        } else {
          wd = word[s];
          pr = pre[s];
        }
        const u64 pos = voff + ebase + pr + (u64)__popcll(wd & below[s / G::SPB]);
        if (pos >= vcap) {  // offsets disagree with the bitmap: never write past the values
          bad = true;
          continue;
        }
        if (j.vbytes == 8)
          ((double*)j.values)[pos] = c[s];
        else
          ((float*)j.values)[pos] = (float)c[s];
      }
    } else {
      if (lane < EPW * W) bm[lane] = 0ull;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int s = 0; s < NS; ++s) G::bitmap_or(bm, ballot(keep[s]), s, ne, lane);
      asm volatile("" ::: "memory");
      // bitmap words out, exclusive word prefixes inside each element
      if (lane < ne * W) {
        const u64 wd = bm[lane];
        gbm[e0 * W + lane] = wd;
        const int ee = lane / W, w = lane % W;
        u32 pre = 0u;
        for (int k = 0; k < w; ++k) pre += (u32)__popcll(bm[ee * W + k]);
        wp[lane] = pre;
        if (w == W - 1) {
          const u64 expect = eptr[e0 + ee + 1] - eptr[e0 + ee];
          if ((u64)(pre + (u32)__popcll(wd)) != expect) bad = true;
        }
      }
      asm volatile("" ::: "memory");
      // kept values at their element offsets
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (!keep[s]) continue;
        const int PI = G::pencil(s, lane), ax = G::axis(s, lane);
        const int ee = PI / G::n2, f = ax * G::n2 + PI % G::n2;
        const int wi = ee * W + (f >> 6);
        const u64 rank = (u64)wp[wi] + (u64)__popcll(bm[wi] & ((1ull << (f & 63)) - 1ull));
        const u64 pos = voff + eptr[e0 + ee] + rank;
        if (pos >= vcap) {  // offsets disagree with the bitmap: never write past the values
          bad = true;
          continue;
        }
        if (j.vbytes == 8)
          ((double*)j.values)[pos] = c[s];
        else
          ((float*)j.values)[pos] = (float)c[s];
      }
    }
    double cm[NS], ut[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) cm[s] = keep[s] ? c[s] : 0.0;
    G::inverse(cm, ut, L.buf[wv], mt, j.tab, lane);
    // quadrature weights of the slots, the same way
    if (j.jac) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        wq[s] = G::valid(s, lane, ne) ? j.jac[e0 + G::elem(s, lane)] * L.tab.w3[s][lane] : 0.0;
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) wq[s] = L.tab.w3[s][lane];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double d = u[s] - ut[s];
      const double x = G::valid(s, lane, ne) ? wq[s] * (d * d) : 0.0;
      if constexpr (EXACT) {
        const double r = xadd_r(ar, PR, x);
        if (r != 0.0) slow_bin(gR, r);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        pr += x;
      }
    }
  }
  if (ballot(bad)) {
    if (lane == 0) atomicOr(&st->flags, ST_LIST);
  }
  if constexpr (!EXACT) {
    const double r = xadd_sum(ar, PR, pr);
    if (r != 0.0) slow_bin(gR, r);
  }
  long long v[3];
  xints(ar, PR, v);
  block_sum_i64<3>(v, L.red, tid);
  if (tid < 3) j.slotsB[((size_t)comp * j.gB + vb) * 4 + tid] = L.red[0][tid];
  if (!tail || !last_block(j.done + D_PASSB * 8 + comp, &L.last, nvb)) return;
  passB_tail(j, comp, L.r3);
}

template <int N, int PREC>
__global__ __launch_bounds__(256, ISR_FAST_MINB) void k_passB(Job j) {
  __shared__ PassBLds<N, PREC> L;
  passB_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

// ---- decompress of blobs made by this engine --------------------------------------
// The blob's kept values go back into the slots pass B took them from, and the
// same inverse runs on them, so that the reconstruction is the one whose
// error pass B measured, bit for bit (FP32 / BF16 blobs).  One tile per
// wavefront, tiles of every component in turn.
template <int N, int PREC>
__global__ __launch_bounds__(256) void k_decompW(Job j, void* out, int out_fp64) {
  typedef Eng<N, PREC> G;
  constexpr int n = G::n, n2 = G::n2, n3 = G::n3, NS = G::NS, EPW = G::EPW, W = G::W;
  static_assert(EPW * W <= 16, "tile bitmap fits the LDS slot");
  __shared__ typename G::wt buf[4][G::LDSW];
  __shared__ u64 bm[4][16];
  __shared__ u32 wp[4][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  const long long E = j.n_elem, tiles = (E + EPW - 1) / EPW, total = tiles * j.ncomp;
  for (long long tk = (long long)blockIdx.x * 4 + wv; tk < total; tk += (long long)gridDim.x * 4) {
    const int comp = (int)(tk / tiles);
    const long long e0 = (tk % tiles) * EPW;
    const int ne = (int)((E - e0) < EPW ? (E - e0) : EPW);
    const u64* gbm = j.bitmap + ((size_t)comp * E + e0) * W;
    const u64* eptr = j.elem_ptr + (size_t)comp * (E + 1);
    const u64 voff = j.voff[comp];
    if (lane < ne * W) bm[wv][lane] = gbm[lane];
    asm volatile("" ::: "memory");
    if (lane < ne * W) {
      const int ee = lane / W, w = lane % W;
      u32 pre = 0u;
      for (int k = 0; k < w; ++k) pre += (u32)__popcll(bm[wv][ee * W + k]);
      wp[wv][lane] = pre;
    }
    asm volatile("" ::: "memory");
    double cm[NS], ut[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      cm[s] = 0.0;
      if (!G::valid(s, lane, ne)) continue;
      const int PI = G::pencil(s, lane), ax = G::axis(s, lane);
      const int ee = PI / n2, f = ax * n2 + PI % n2, wi = ee * W + (f >> 6);
      const u64 wd = bm[wv][wi];
      if ((wd >> (f & 63)) & 1ull) {
        const u64 pos = voff + eptr[e0 + ee] + wp[wv][wi] + (u64)__popcll(wd & ((1ull << (f & 63)) - 1ull));
        cm[s] = j.vbytes == 8 ? ((const double*)j.values)[pos] : (double)((const float*)j.values)[pos];
      }
    }
    G::inverse(cm, ut, buf[wv], mt, j.tab, lane);
    const size_t ob = ((size_t)comp * E + e0) * n3;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!G::valid(s, lane, ne)) continue;
      const size_t o = ob + (size_t)G::pencil(s, lane) * n + G::axis(s, lane);
      if (out_fp64)
        ((double*)out)[o] = ut[s];
      else
        ((float*)out)[o] = (float)ut[s];
    }
  }
}

// ---- launchers ------------------------------------------------------------------
#define ISR_FAST_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int PREC>
hipError_t launch_decompW_prec(const Job& j, int gx, hipStream_t s, void* out, int out_fp64) {
  switch (j.order) {
#define CASE(NN)                                                                       \
  case NN:                                                                             \
    hipLaunchKernelGGL((k_decompW<NN, PREC>), dim3(gx), dim3(256), 0, s, j, out, out_fp64); \
    break;
    ISR_FAST_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_fast_prec(int kind, const Job& j, int gx, hipStream_t s) {
  const dim3 grid(gx, j.ncomp), blk(256);
  switch (j.order) {
#define CASE(NN)                                                   \
  case NN:                                                         \
    if (kind == F_SAMPLE)                                          \
      hipLaunchKernelGGL((k_sample<NN, PREC>), grid, blk, 0, s, j); \
    else if (kind == F_PASSA)                                      \
      hipLaunchKernelGGL((k_passA<NN, PREC>), grid, blk, 0, s, j);  \
    else if (kind == F_PASSB)                                      \
      hipLaunchKernelGGL((k_passB<NN, PREC>), grid, blk, 0, s, j);  \
    else                                                           \
      return hipErrorInvalidValue;                                 \
    break;
    ISR_FAST_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
int resident_fast_prec(int kind, int order) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (order) {
#define CASE(NN)                                                                                         \
  case NN:                                                                                               \
    if (kind == F_SAMPLE)                                                                                \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_sample<NN, PREC>, 256, 0);   \
    else if (kind == F_PASSA)                                                                            \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passA<NN, PREC>, 256, 0);    \
    else if (kind == F_PASSB)                                                                            \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passB<NN, PREC>, 256, 0);    \
    break;
    ISR_FAST_ORDERS(CASE)
#undef CASE
    default:
      break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 2;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace isr
