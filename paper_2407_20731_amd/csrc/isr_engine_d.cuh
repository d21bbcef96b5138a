// Dense-tile streaming path for the MFMA precisions (FP32, BF16 split).
//
// A wavefront owns a tile of T consecutive elements, T n^3 field values that
// are contiguous in HBM.  Everything that is done once per value (norm and
// error terms, energies, window tests, keep decisions, bitmaps, ranks) runs
// on the dense order v = 64 s + lane, s = 0..S-1, so that no lane idles on
// padding; only the three contractions see padded shapes.  The tile lives in
// a per-wave LDS buffer in FP32, flat in (element, k, j, i) order, and each
// contraction runs in place, block by block:
//
//   forward  along i (stride 1), j (stride n), k (stride n^2) with A,
//   inverse  along k, j, i with V,
//
// after which the buffer holds the coefficients in (element, r, q, p) order,
// which is the flat coefficient index f = p + n q + n^2 r of every element:
// the dense slot of a value is its position in the blob order as well.
//
// One 16x16 MFMA tile contracts 16 NCOPY pencils: for n <= 8 the A operand
// holds two block-diagonal 8x8 copies of the 1D matrix (two sets of 16
// pencils pair up along K), for 9 <= n <= 16 one 16x16 copy (K padded to 16).
// Lane l = 16 g + P holds pencil PB b + 16 (g / GPC) + P of block b and
// indices 4 (g % GPC) + m, m = 0..3, in its four input and output registers.
// Pencils of a stage partition the tile, so a block reads and writes only its
// own positions and in-place stages need no barrier.
#pragma once

#include "isr_engine_l.cuh"

// Minimum resident workgroups per CU the dense-tile passes are compiled for.
#ifndef ISR_DENSE_MINB
#define ISR_DENSE_MINB 3
#endif
// Blocks of one contraction kept in flight (independent LDS -> MFMA -> LDS chains).
#ifndef ISR_DENSE_UNROLL
#define ISR_DENSE_UNROLL 2
#endif


namespace isr {

template <int N, int PREC, int T>
struct EngD {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static_assert(PREC != P_FP64 && n >= 2 && n <= 12 && T >= 1, "dense-tile engine: MFMA paths, orders 1..11");
  static constexpr int KP = n <= 8 ? 8 : 16;   // padded length of one copy of the 1D matrix
  static constexpr int NCOPY = 16 / KP;        // copies in a 16x16 tile
  static constexpr int GPC = 4 / NCOPY;        // lane groups of 16 per copy
  static constexpr int PB = 16 * NCOPY;        // pencils per block
  static constexpr int TP = T * n2;            // pencils per tile and stage
  static constexpr int NB = (TP + PB - 1) / PB;
  static constexpr int TV = T * n3;            // values per tile
  static constexpr int S = (TV + 63) / 64;     // dense slots per lane
  static constexpr int LDSW = S * 64;          // floats of the dense slots
  // In the passes (UM = true) rows of the contracted index past n (a0 + m >=
  // n, when KP > n) are read without a lane mask: the A operand's columns
  // there are zero, so whatever finite value sits at such an address adds
  // nothing, and the lane-mask updates around every masked load go away.
  // The farthest such read (the last pencil along k) ends before LDSB; the
  // buffer's tail past the dense slots is zeroed once per kernel.  Stores
  // stay masked.  The sample pass keeps masked loads and the smaller buffer
  // (its occupancy is bound by LDS at n = 10).
  static constexpr int OVR = T * n3 + n2 * (KP > n ? KP - n : 0);
  static constexpr int LDSB = ((OVR > LDSW ? OVR : LDSW) + 63) / 64 * 64;  // floats of the wave buffer
  static constexpr int W = (n3 + 63) / 64;     // bitmap words per element
  static_assert(S <= 32, "dense slots per lane");
  // window candidates staged per wave in pass A (n >= 9: half, so that the
  // larger tables leave room for four workgroups per CU), and the workgroups
  // per CU pass B is compiled for (n <= 7: four, 128 VGPRs, measured faster
  // than three without spills)
  static constexpr int CAPB = n >= 9 ? 128 : 256;
  static constexpr int MINB_B = n <= 7 ? 4 : ISR_DENSE_MINB;  // (dense_minb_b below)

  struct Mats {
    float fa[4], fv[4];  // FP32 A-operand fragments (forward A, inverse V)
    s4 ha, la, hv, lv;   // BF16 hi / lo fragments
  };

  // A fragment of lane (row, g): element (row, K = 4 g + v) of the 16x16
  // operand, the 1D matrix on the diagonal copies and zero elsewhere.
  static DEV void frag(float (&f)[4], s4& h, s4& l, const float* M, int lane) {
    const int row = lane & 15, g = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int K = 4 * g + v;
      const int o = row % KP, a = K % KP;
      const bool on = (row / KP) == (K / KP) && o < n && a < n;
      const float m = on ? M[o * n + a] : 0.0f;
      f[v] = m;
      const short hi = to_bf16(m);
      h[v] = hi;
      l[v] = to_bf16(m - from_bf16(hi));
    }
  }
  static DEV void init(Mats& mt, const DevTables& t, int lane) {
    frag(mt.fa, mt.ha, mt.la, t.A32, lane);
    frag(mt.fv, mt.hv, mt.lv, t.V32, lane);
  }

  // One 16x16 tile: out[o][pencil] = sum_a M[o][a] x[a][pencil].
  static DEV void mfma(const float (&x)[4], float (&y)[4], const float (&f)[4], s4 h, s4 l) {
    f4 d = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (PREC == P_FP32) {
#pragma unroll
      for (int s = 0; s < 4; ++s) d = __builtin_amdgcn_mfma_f32_16x16x4f32(f[s], x[s], d, 0, 0, 0);
    } else {
      s4 xh, xl;
      split_bf16x4(x[0], x[1], x[2], x[3], xh, xl);
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, xh, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(l, xh, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, xl, d, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) y[v] = d[v];
  }

  // Flat position of index 0 of pencil PI along axis AX (0: i, 1: j, 2: k).
  template <int AX>
  static DEV int pbase(int PI) {
    if constexpr (AX == 0) return PI * n;                    // pencil (e, k, j)
    if constexpr (AX == 1) return (PI / n) * n2 + PI % n;    // pencil (e, k, i)
    return (PI / n2) * n3 + PI % n2;                         // pencil (e, j, i)
  }
  template <int AX>
  static constexpr int stride() {
    return AX == 0 ? 1 : (AX == 1 ? n : n2);
  }

  // In-place contraction of every pencil of the tile along AX.
  template <int AX, bool UM>
  static DEV void stage(float* buf, const float (&f)[4], s4 h, s4 l, int lane) {
    constexpr int ST = stride<AX>();
    const int P = lane & 15, g = lane >> 4;
    const int hc = g / GPC, a0 = 4 * (g % GPC);
#pragma unroll ISR_DENSE_UNROLL
    for (int b = 0; b < NB; ++b) {
      const int PI = PB * b + 16 * hc + P;
      const bool pv = PI < TP;
      float* p = buf + (pv ? pbase<AX>(PI) + a0 * ST : 0);
      float x[4], y[4];
      if constexpr (AX == 0 && n % 2 == 0) {
        // contiguous pairs of one pencil: 8-byte accesses (even n keeps them
        // aligned and a pair either inside or outside the pencil)
        typedef float fl2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int m = 0; m < 4; m += 2) {
          const fl2 z = (UM || (pv && a0 + m < n)) ? *(const fl2*)(p + m) : fl2{0.0f, 0.0f};
          x[m] = z.x;
          x[m + 1] = z.y;
        }
        mfma(x, y, f, h, l);
#pragma unroll
        for (int m = 0; m < 4; m += 2)
          if (pv && a0 + m < n) *(fl2*)(p + m) = fl2{y[m], y[m + 1]};
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = (UM || (pv && a0 + m < n)) ? p[m * ST] : 0.0f;
        mfma(x, y, f, h, l);
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if (pv && a0 + m < n) p[m * ST] = y[m];
      }
    }
    asm volatile("" ::: "memory");
  }
  // Zero the wave buffer's tail past the dense slots (once per kernel, before
  // the first contraction).
  static DEV void clear_tail(float* buf, int lane) {
    for (int i = LDSW + lane; i < LDSB; i += 64) buf[i] = 0.0f;
  }
  template <bool UM = true>
  static DEV void forward(float* buf, const Mats& mt, int lane) {
    asm volatile("" ::: "memory");
    stage<0, UM>(buf, mt.fa, mt.ha, mt.la, lane);
    stage<1, UM>(buf, mt.fa, mt.ha, mt.la, lane);
    stage<2, UM>(buf, mt.fa, mt.ha, mt.la, lane);
  }
  static DEV void inverse(float* buf, const Mats& mt, int lane) {
    asm volatile("" ::: "memory");
    stage<2, true>(buf, mt.fv, mt.hv, mt.lv, lane);
    stage<1, true>(buf, mt.fv, mt.hv, mt.lv, lane);
    stage<0, true>(buf, mt.fv, mt.hv, mt.lv, lane);
  }
};

// pass B launch bound of order N (the kernel attribute takes no template-id)
template <int N>
constexpr int dense_minb_b() {
  return N + 1 <= 7 ? 4 : ISR_DENSE_MINB;
}

// pass A launch bound of shape (N, T): four workgroups per CU (at most 128
// VGPRs) at N = 5 with tiles of up to two elements, measured 10 % faster there
// than three; larger shapes spill at 128, and two workgroups at N = 9
// measured 12 % slower than three
template <int N, int T>
constexpr int dense_minb_a() {
  return (N == 5 && T <= 2) ? 4 : ISR_DENSE_MINB;
}

// Element (within the tile) and flat index of dense position v (positions
// past the tile, which are masked out, keep f inside the tables).
template <class G>
DEV void dense_ef(int v, int& e, int& f) {
  if constexpr (G::TV == G::n3) {
    e = 0;
    f = v < G::n3 ? v : G::n3 - 1;
  } else {
    e = v / G::n3;
    f = v - e * G::n3;
  }
}

// ---- sample pass --------------------------------------------------------------
template <int N, int PREC, int T>
struct SampleLdsD {
  float buf[4][EngD<N, PREC, T>::LDSW];
  TabLdsL<EngD<N, PREC, T>::n3> tab;
  u32 hc[SBINS];
  float hs[SBINS];  // sums of energy / 2^(bin exponent), each term in [1, 2)
  double u2[4];
  int maxe;
  int last;
};

template <int N, int PREC, int T>
DEV void sampleD_body(const Job& j, int comp, int vb, int nvb, SampleLdsD<N, PREC, T>& L, bool tail) {
  typedef EngD<N, PREC, T> G;
  constexpr int n3 = G::n3, S = G::S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  for (int k = tid; k < SBINS; k += 256) {
    L.hc[k] = 0u;
    L.hs[k] = 0.0f;
  }
  if (tid == 0) L.maxe = 0;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tabl_load(L.tab, j.tab, tid);
  __syncthreads();
  const long long E = j.n_elem, tiles = (E + T - 1) / T;
  const long long ss = j.sample_stride > 0 ? j.sample_stride : 1;
  const long long stiles = (tiles + ss - 1) / ss;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const long long nw = (long long)nvb * 4;
  float* buf = L.buf[wv];
  double u2 = 0.0;
  int maxe = 0;
  for (long long k = (long long)vb * 4 + wv; k < stiles; k += nw) {
    const long long e0 = k * ss * T;
    const int nv = (int)((E - e0) < T ? (E - e0) : T) * n3;
    const double* tile = ub + e0 * n3;
    // every load of the tile issued before any is used (one memory latency
    // per tile instead of one per slot)
    double ut[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      // every lane loads (from inside the tile), then masks: no branch per slot
      const double lv = __builtin_nontemporal_load(tile + (v < nv ? v : nv - 1));
      ut[s] = v < nv ? lv : 0.0;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const double u = ut[s];
      if (v < nv) {
        const double x = (j.jac ? j.jac[e0 + e] * L.tab.w3[f] : L.tab.w3[f]) * (u * u);
        u2 += x;
        const int ex = bits_exp(dbits(x));
        maxe = ex > maxe ? ex : maxe;
      }
      buf[v] = (float)u;
    }
    G::template forward<false>(buf, mt, lane);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      if (v >= nv) continue;
      int e, f;
      dense_ef<G>(v, e, f);
      const double c = (double)buf[v];
      const double en = (j.jac ? j.jac[e0 + e] * L.tab.g3[f] : L.tab.g3[f]) * (c * c);
      const int b = bits_exp(dbits(en));
      if (b < HBINS - 1) {  // rounded sums only place the window
        atomicAdd(&L.hc[b], 1u);
        atomicAdd(&L.hs[b], (float)ldexp(en, 1023 - b));
      }
    }
    asm volatile("" ::: "memory");
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

template <int N, int PREC, int T>
__global__ __launch_bounds__(256, ISR_DENSE_MINB) void k_sampleD(Job j) {
  __shared__ SampleLdsD<N, PREC, T> L;
  sampleD_body<N, PREC, T>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

// ---- pass A ---------------------------------------------------------------------
template <int N, int PREC, int T>
struct PassALdsD {
  float buf[4][EngD<N, PREC, T>::LDSB];
  TabLdsL<EngD<N, PREC, T>::n3> tab;
  u64 key[4][EngD<N, PREC, T>::CAPB];
  u32 idx[4][EngD<N, PREC, T>::CAPB];
  u32 ecnt[4][T];
  long long red[4][8];
};

template <int N, int PREC, int T>
DEV void passAD_body(const Job& j, int comp, int vb, int nvb, PassALdsD<N, PREC, T>& L) {
  typedef EngD<N, PREC, T> G;
  constexpr int n3 = G::n3, S = G::S;
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
  const long long E = j.n_elem, tiles = (E + T - 1) / T;
  u32* cnt = j.cnt + (size_t)comp * E;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tabl_load(L.tab, j.tab, tid);
  __syncthreads();
  XAcc an = {0.0, 0.0, 0.0}, ae = {0.0, 0.0, 0.0};
  double pe = 0.0;  // fixed-order sum of the energies below the window
  double pn = 0.0;  // fixed-order sum of the norm terms
  u64 hi_tot = 0ull;
  u32 ncap = 0u;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const long long nw = (long long)nvb * 4;
  float* buf = L.buf[wv];
  G::clear_tail(buf, lane);
  for (long long t = (long long)vb * 4 + wv; t < tiles; t += nw) {
    const long long e0 = t * T;
    const int ne = (int)((E - e0) < T ? (E - e0) : T), nv = ne * n3;
    const double* tile = ub + e0 * n3;
    // field values in (every load of the tile issued before the first is
    // used: one memory latency per tile), norm terms on the way
    double ut[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      // every lane loads (from inside the tile), then masks: no branch per slot
      const double lv = __builtin_nontemporal_load(tile + (v < nv ? v : nv - 1));
      ut[s] = v < nv ? lv : 0.0;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const double u = ut[s];
      pn += v < nv ? (j.jac ? j.jac[e0 + e] * L.tab.w3[f] : L.tab.w3[f]) * (u * u) : 0.0;
      buf[v] = (float)u;
    }
    G::forward(buf, mt, lane);
    if constexpr (T > 1) {
      if (lane < T) L.ecnt[wv][lane] = 0u;
      asm volatile("" ::: "memory");
    }
    u32 hc = 0u;
#pragma unroll 2
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const bool ok = v < nv;
      const double c = (double)buf[v];
      const double en = ok ? (j.jac ? j.jac[e0 + e] * L.tab.g3[f] : L.tab.g3[f]) * (c * c) : 0.0;
      const u64 key = dbits(en);
      const int ex = bits_exp(key);
      const bool hi = ok && ex >= whi;
      const bool cp = ok && ex < whi && ex >= wlo;
      pe += (ok && ex < wlo) ? en : 0.0;
      if (hi && ex == HBINS - 1) slow_bin(gE, en);  // Inf/NaN: counted in the flag bin
      const u64 bh = ballot(hi);
      hc += (u32)__popcll(bh);
      if constexpr (T > 1) {
        if (hi) atomicAdd(&L.ecnt[wv][e], 1u);
      }
      const u64 bc = ballot(cp);
      if (bc) {
        const u32 pos = ncap + (u32)__popcll(bc & ((1ull << lane) - 1ull));
        if (cp) {
          L.key[wv][pos] = key;
          L.idx[wv][pos] = (u32)(e0 + e);
        }
        ncap += (u32)__popcll(bc);
        if (ncap > (u32)(G::CAPB - 64)) {
          asm volatile("" ::: "memory");
          cap_flush(L.key[wv], L.idx[wv], ncap, st, list, lidx, j.list_cap, lane);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    hi_tot += hc;
    if constexpr (T == 1) {
      if (lane == 0) cnt[e0] = hc;
    } else {
      asm volatile("" ::: "memory");
      if (lane < ne) cnt[e0 + lane] = L.ecnt[wv][lane];
    }
    asm volatile("" ::: "memory");
  }
  asm volatile("" ::: "memory");
  cap_flush(L.key[wv], L.idx[wv], ncap, st, list, lidx, j.list_cap, lane);
  {
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

template <int N, int PREC, int T>
__global__ __launch_bounds__(256, (dense_minb_a<N, T>())) void k_passAD(Job j) {
  __shared__ PassALdsD<N, PREC, T> L;
  passAD_body<N, PREC, T>(j, blockIdx.y, blockIdx.x, gridDim.x, L);
}

// ---- pass B ---------------------------------------------------------------------
template <int N, int PREC, int T>
struct PassBLdsD {
  float buf[4][EngD<N, PREC, T>::LDSB];
  TabLdsL<EngD<N, PREC, T>::n3> tab;
  u64 bal[4][EngD<N, PREC, T>::S + 1];
  u32 wc[4][T * EngD<N, PREC, T>::W];
  long long red[4][8];
  __int128 r3[4][3];
  int last;
};

template <int N, int PREC, int T>
DEV void passBD_body(const Job& j, int comp, int vb, int nvb, PassBLdsD<N, PREC, T>& L, bool tail) {
  typedef EngD<N, PREC, T> G;
  constexpr int n3 = G::n3, S = G::S, W = G::W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const XParm PR = xparm(st->xm_err, j.xh);
  HistBin* gR = j.histR + (size_t)comp * HBINS;
  const u64 tk = dbits(st->tau);
  u64 voff = 0ull;
  for (int cc = 0; cc < comp; ++cc) voff += j.st[cc].kept;
  const u64 vcap = (u64)j.ncomp * (u64)j.n_elem * (u64)n3;
  const long long E = j.n_elem, tiles = (E + T - 1) / T;
  const u64* eptr = j.elem_ptr + (size_t)comp * (E + 1);
  u64* gbm = j.bitmap + (size_t)comp * E * W;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  tabl_load(L.tab, j.tab, tid);
  __syncthreads();
  XAcc ar = {0.0, 0.0, 0.0};
  double pr = 0.0;  // fixed-order sum of the error terms
  bool bad = false;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const long long nw = (long long)nvb * 4;
  float* buf = L.buf[wv];
  G::clear_tail(buf, lane);
  u64* bal = L.bal[wv];
  const u64 lt = (1ull << lane) - 1ull;
  for (long long t = (long long)vb * 4 + wv; t < tiles; t += nw) {
    const long long e0 = t * T;
    const int ne = (int)((E - e0) < T ? (E - e0) : T), nv = ne * n3;
    const double* tile = ub + e0 * n3;
    double ur[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      // every lane loads (from inside the tile), then masks: no branch per slot
      const double lv = __builtin_nontemporal_load(tile + (v < nv ? v : nv - 1));
      ur[s] = v < nv ? lv : 0.0;
      buf[v] = (float)ur[s];
    }
    G::forward(buf, mt, lane);
    // keep decisions in dense order: the tile's kept values are contiguous in
    // the blob from elem_ptr[e0] on, in this very order
    const u64 base = voff + eptr[e0];
    u32 cum = 0u;
    u64 mine = 0ull;
#pragma unroll 2
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const bool ok = v < nv;
      const float cf = buf[v];
      const double c = (double)cf;
      const double en = ok ? (j.jac ? j.jac[e0 + e] * L.tab.g3[f] : L.tab.g3[f]) * (c * c) : 0.0;
      const bool keep = ok && dbits(en) >= tk;
      const u64 bk = ballot(keep);
      if (keep) {
        const u64 pos = base + cum + (u64)__popcll(bk & lt);
        if (pos < vcap) {
          if (j.vbytes == 8)
            ((double*)j.values)[pos] = c;
          else
            ((float*)j.values)[pos] = cf;
        } else {  // offsets disagree with the bitmap: never write past the values
          bad = true;
        }
      }
      buf[v] = keep ? cf : 0.0f;
      if constexpr (T == 1) {
        mine = lane == s ? bk : mine;
      } else {
        if (lane == 0) bal[s] = bk;
      }
      cum += (u32)__popcll(bk);
      __builtin_amdgcn_sched_barrier(0);
    }
    // bitmap words and the per-element counts against elem_ptr
    if constexpr (T == 1) {
      if (lane < W) gbm[e0 * W + lane] = mine;
      if ((u64)cum != eptr[e0 + 1] - eptr[e0]) bad = true;
    } else {
      if (lane == 0) bal[S] = 0ull;
      asm volatile("" ::: "memory");
      for (int L0 = lane; L0 < ne * W; L0 += 64) {
        const int e = L0 / W, w = L0 - e * W;
        const int o = e * n3 + 64 * w, sl = o >> 6, r = o & 63;
        u64 wd = bal[sl];
        if (r) wd = (wd >> r) | (bal[sl + 1] << (64 - r));
        const int len = n3 - 64 * w;
        if (len < 64) wd &= (1ull << len) - 1ull;
        gbm[e0 * W + L0] = wd;
        L.wc[wv][L0] = (u32)__popcll(wd);
      }
      asm volatile("" ::: "memory");
      if (lane < ne) {
        u32 k = 0u;
        for (int w = 0; w < W; ++w) k += L.wc[wv][lane * W + w];
        if ((u64)k != eptr[e0 + lane + 1] - eptr[e0 + lane]) bad = true;
      }
      asm volatile("" ::: "memory");
    }
    G::inverse(buf, mt, lane);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const double d = ur[s] - (double)buf[v];
      pr += v < nv ? (j.jac ? j.jac[e0 + e] * L.tab.w3[f] : L.tab.w3[f]) * (d * d) : 0.0;
    }
    asm volatile("" ::: "memory");
  }
  if (ballot(bad)) {
    if (lane == 0) atomicOr(&st->flags, ST_LIST);
  }
  {
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

template <int N, int PREC, int T>
__global__ __launch_bounds__(256, dense_minb_b<N>()) void k_passBD(Job j) {
  __shared__ PassBLdsD<N, PREC, T> L;
  passBD_body<N, PREC, T>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

// ---- decompress of blobs made by this engine --------------------------------------
// Kept values back into the dense slots (a tile's kept values are contiguous
// in the blob in dense order), zeros elsewhere, and pass B's inverse on the
// same buffer: the reconstruction pass B measured, bit for bit.
template <int N, int PREC, int T>
__global__ __launch_bounds__(256) void k_decompD(Job j, void* out, int out_fp64) {
  typedef EngD<N, PREC, T> G;
  constexpr int n3 = G::n3, S = G::S, W = G::W;
  __shared__ float bufs[4][G::LDSB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  float* buf = bufs[wv];
  G::clear_tail(buf, lane);
  const u64 lt = (1ull << lane) - 1ull;
  const long long E = j.n_elem, tiles = (E + T - 1) / T, total = tiles * j.ncomp;
  for (long long tk = (long long)blockIdx.x * 4 + wv; tk < total; tk += (long long)gridDim.x * 4) {
    const int comp = (int)(tk / tiles);
    const long long e0 = (tk % tiles) * T;
    const int ne = (int)((E - e0) < T ? (E - e0) : T), nv = ne * n3;
    const u64* gbm = j.bitmap + (size_t)comp * E * W;
    const u64 base = j.voff[comp] + j.elem_ptr[(size_t)comp * (E + 1) + e0];
    u32 cum = 0u;
#pragma unroll 2
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      int e, f;
      dense_ef<G>(v, e, f);
      const bool keep = v < nv && ((gbm[(size_t)(e0 + e) * W + (f >> 6)] >> (f & 63)) & 1ull);
      const u64 bk = ballot(keep);
      float val = 0.0f;
      if (keep) {
        const u64 pos = base + cum + (u64)__popcll(bk & lt);
        val = j.vbytes == 8 ? (float)((const double*)j.values)[pos] : ((const float*)j.values)[pos];
      }
      buf[v] = val;
      cum += (u32)__popcll(bk);
    }
    asm volatile("" ::: "memory");
    G::inverse(buf, mt, lane);
    const size_t ob = ((size_t)comp * E + e0) * n3;
#pragma unroll 2
    for (int s = 0; s < S; ++s) {
      const int v = 64 * s + lane;
      if (v >= nv) continue;
      if (out_fp64)
        ((double*)out)[ob + v] = (double)buf[v];
      else
        ((float*)out)[ob + v] = buf[v];
    }
    asm volatile("" ::: "memory");
  }
}

// ---- launchers ------------------------------------------------------------------
template <int PREC>
hipError_t launch_decompD_prec(const Job& j, int gx, hipStream_t s, void* out, int out_fp64) {
#define CASE(O, T)                                                                       \
  if (j.order == O && j.tile == T) {                                                     \
    hipLaunchKernelGGL((k_decompD<O, PREC, T>), dim3(gx), dim3(256), 0, s, j, out, out_fp64); \
    return hipGetLastError();                                                            \
  }
  ISR_DENSE_SHAPES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_dense_prec(int kind, const Job& j, int gx, hipStream_t s) {
  const dim3 grid(gx, j.ncomp), blk(256);
#define CASE(O, T)                                                     \
  if (j.order == O && j.tile == T) {                                   \
    if (kind == F_SAMPLE)                                              \
      hipLaunchKernelGGL((k_sampleD<O, PREC, T>), grid, blk, 0, s, j); \
    else if (kind == F_PASSA)                                          \
      hipLaunchKernelGGL((k_passAD<O, PREC, T>), grid, blk, 0, s, j);  \
    else if (kind == F_PASSB)                                          \
      hipLaunchKernelGGL((k_passBD<O, PREC, T>), grid, blk, 0, s, j);  \
    else                                                               \
      return hipErrorInvalidValue;                                     \
    return hipGetLastError();                                          \
  }
  ISR_DENSE_SHAPES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <int PREC>
int resident_dense_prec(int kind, int order, int tile) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define CASE(O, T)                                                                                          \
  if (order == O && tile == T) {                                                                            \
    if (kind == F_SAMPLE)                                                                                   \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_sampleD<O, PREC, T>, 256, 0);   \
    else if (kind == F_PASSA)                                                                               \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passAD<O, PREC, T>, 256, 0);    \
    else if (kind == F_PASSB)                                                                               \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passBD<O, PREC, T>, 256, 0);    \
  }
  ISR_DENSE_SHAPES(CASE)
#undef CASE
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace isr
