// Streaming path for orders 8..11 on MFMA (FP32, BF16 split): one element per
// wavefront.  The element is loaded with coalesced 8-byte loads (norm terms
// taken on the way) into a per-wave LDS copy in FP32; every contraction then
// runs block by block over 16-pencil blocks (the MFMA columns), the
// contracted index padded to 16 (the K of one tile), reading and writing the
// same LDS positions in place:
//
//   forward  i (pattern 1 -> 1), j (2 -> 2), k (3 -> registers)
//   inverse  r (registers -> 3), q (2 -> 2), p (1 -> registers)
//
// with the LDS coordinates of a (pencil (a, b), index ax) pair being
// (a, b, ax), (a, ax, b) and (ax, a, b) for patterns 1, 2, 3.  A block only
// touches the positions of its own pencils, so in-place stages are safe.
// Lane l = 16 g + P of block b holds pencil 16 b + P and indices 4 g + m,
// m = 0..3.  The kept values are staged in LDS by flat index and written in
// rank order once the element's bitmap is complete.  (Orders 12..15 would need
// more LDS per wavefront than fits four of them; they run the general passes.)
#pragma once

#include "isr_engine.cuh"

namespace isr {

template <int N, int PREC>
struct EngL {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static_assert(n >= 9 && n <= 12 && PREC != P_FP64, "large-order engine: MFMA paths, orders 8..11");
  static constexpr int NB = (n2 + 15) / 16;  // pencil blocks per element
  static constexpr int P0 = n + 1;           // LDS row pitch (floats)
  static constexpr int LDSW = n * n * P0;
  static constexpr int W = (n3 + 63) / 64;   // bitmap words per element
  static constexpr int CH = 16;              // field values per lane per load chunk
  static constexpr int NCH = (n3 + 64 * CH - 1) / (64 * CH);

  struct Mats {
    float fa[4], fv[4];
    s4 ha, la, hv, lv;
  };

  DEV static int pencil(int b, int lane) { return 16 * b + (lane & 15); }
  DEV static int axis(int m, int lane) { return 4 * (lane >> 4) + m; }
  DEV static bool valid(int b, int m, int lane) { return pencil(b, lane) < n2 && axis(m, lane) < n; }

  static DEV void frag(float (&f)[4], s4& h, s4& l, const float* M, int lane) {
    const int row = lane & 15, g = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 4 * g + v;
      const float m = (row < n && a < n) ? M[row * n + a] : 0.0f;
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

  // One 16x16 tile: out[b][pencil] = sum_a M[b][a] x[a][pencil].
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

  template <int PAT>
  static DEV int addr(int PI, int ax) {
    const int a = PI / n, b = PI % n;
    const int x2 = PAT == 3 ? ax : a;
    const int x1 = PAT == 1 ? b : (PAT == 2 ? ax : a);
    const int x0 = PAT == 1 ? ax : b;
    return (x2 * n + x1) * P0 + x0;
  }
  template <int PAT>
  static DEV void rd(const float* buf, int b, float (&x)[4], int lane) {
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = valid(b, m, lane) ? buf[addr<PAT>(pencil(b, lane), axis(m, lane))] : 0.0f;
  }
  template <int PAT>
  static DEV void wr(float* buf, int b, const float (&y)[4], int lane) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (valid(b, m, lane)) buf[addr<PAT>(pencil(b, lane), axis(m, lane))] = y[m];
  }
  // In-place stage over every block: read pattern RP, contract, write WP.
  template <int PAT>
  static DEV void stage(float* buf, const float (&f)[4], s4 h, s4 l, int lane) {
#pragma unroll 1
    for (int b = 0; b < NB; ++b) {
      float x[4], y[4];
      rd<PAT>(buf, b, x, lane);
      mfma(x, y, f, h, l);
      wr<PAT>(buf, b, y, lane);
    }
    asm volatile("" ::: "memory");
  }

  // Field values of chunk ch: lane holds value q = 64 (ch CH + it) + lane.
  static DEV void load_chunk(const double* __restrict__ tile, int ch, double (&r)[CH], int lane) {
#pragma unroll
    for (int it = 0; it < CH; ++it) {
      const int q = 64 * (ch * CH + it) + lane;
      r[it] = q < n3 ? __builtin_nontemporal_load(tile + q) : 0.0;
    }
  }
  // value q = (k n + j) n + i -> pattern-1 position of pencil (k, j), index i
  static DEV int pos1(int q) { return (q / n) * P0 + q % n; }
};

// w3 and g3 of one order (n^3 doubles each) in LDS
template <int NN3>
struct TabLdsL {
  double w3[NN3], g3[NN3];
};
template <int NN3>
DEV void tabl_load(TabLdsL<NN3>& T, const DevTables& t, int tid) {
  for (int k = tid; k < NN3; k += 256) {
    T.w3[k] = t.w3[k];
    T.g3[k] = t.g3[k];
  }
}

template <int N, int PREC>
struct SampleLdsL {
  float buf[4][EngL<N, PREC>::LDSW];
  TabLdsL<EngL<N, PREC>::n3> tab;
  u32 hc[SBINS];
  float hs[SBINS];  // sums of energy / 2^(bin exponent), each term in [1, 2)
  double u2[4];
  int maxe;
  int last;
};

// Forward transform of element e (field tile at `tile`) into buf; the norm
// terms of its values go to `norm(q, x)` on the way.
template <class G, class F>
DEV void fwd_l(const double* tile, float* buf, const typename G::Mats& mt, int lane, F norm) {
#pragma unroll 1
  for (int ch = 0; ch < G::NCH; ++ch) {
    double r[G::CH];
    G::load_chunk(tile, ch, r, lane);
#pragma unroll
    for (int it = 0; it < G::CH; ++it) {
      const int q = 64 * (ch * G::CH + it) + lane;
      if (q < G::n3) {
        norm(q, r[it]);
        buf[G::pos1(q)] = (float)r[it];
      }
    }
  }
  asm volatile("" ::: "memory");
  G::template stage<1>(buf, mt.fa, mt.ha, mt.la, lane);
  G::template stage<2>(buf, mt.fa, mt.ha, mt.la, lane);
}

template <int N, int PREC>
DEV void sampleL_body(const Job& j, int comp, int vb, int nvb, SampleLdsL<N, PREC>& L, bool tail) {
  typedef EngL<N, PREC> G;
  constexpr int n2 = G::n2, n3 = G::n3;
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
  const long long E = j.n_elem;
  const long long ss = j.sample_stride > 0 ? j.sample_stride : 1;
  const long long stiles = (E + ss - 1) / ss;
  const double* ub = j.u + (size_t)comp * j.comp_stride;
  const long long nw = (long long)nvb * 4;
  double u2 = 0.0;
  int maxe = 0;
  float* buf = L.buf[wv];
  for (long long k = (long long)vb * 4 + wv; k < stiles; k += nw) {
    const long long e = k * ss;
    const double jac = j.jac ? j.jac[e] : 1.0;
    fwd_l<G>(ub + e * n3, buf, mt, lane, [&](int q, double x) {
      const double t = (j.jac ? jac * L.tab.w3[q] : L.tab.w3[q]) * (x * x);
      u2 += t;
      const int ex = bits_exp(dbits(t));
      maxe = ex > maxe ? ex : maxe;
    });
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float x[4], y[4];
      G::template rd<3>(buf, b, x, lane);
      G::mfma(x, y, mt.fa, mt.ha, mt.la);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (!G::valid(b, m, lane)) continue;
        const int f = G::axis(m, lane) * n2 + G::pencil(b, lane);
        const double c = (double)y[m];
        const double en = (j.jac ? jac * L.tab.g3[f] : L.tab.g3[f]) * (c * c);
        const int bb = bits_exp(dbits(en));
        if (bb < HBINS - 1) {
          atomicAdd(&L.hc[bb], 1u);
          atomicAdd(&L.hs[bb], (float)ldexp(en, 1023 - bb));
        }
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
__global__ __launch_bounds__(256, 2) void k_sampleL(Job j) {
  __shared__ SampleLdsL<N, PREC> L;
  sampleL_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

template <int N, int PREC>
struct PassALdsL {
  float buf[4][EngL<N, PREC>::LDSW];
  TabLdsL<EngL<N, PREC>::n3> tab;
  u64 key[4][CAPB];
  u32 idx[4][CAPB];
  long long red[4][8];
};

template <int N, int PREC>
DEV void passAL_body(const Job& j, int comp, int vb, int nvb, PassALdsL<N, PREC>& L) {
  typedef EngL<N, PREC> G;
  constexpr int n2 = G::n2, n3 = G::n3;
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
  const long long E = j.n_elem;
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
  for (long long e = (long long)vb * 4 + wv; e < E; e += nw) {
    const double jac = j.jac ? j.jac[e] : 1.0;
    fwd_l<G>(ub + e * n3, buf, mt, lane,
             [&](int q, double x) { pn += (j.jac ? jac * L.tab.w3[q] : L.tab.w3[q]) * (x * x); });
    u32 hc = 0u;
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float x[4], y[4];
      G::template rd<3>(buf, b, x, lane);
      G::mfma(x, y, mt.fa, mt.ha, mt.la);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool v = G::valid(b, m, lane);
        const int f = G::axis(m, lane) * n2 + G::pencil(b, lane);
        const double c = (double)y[m];
        const double en = v ? (j.jac ? jac * L.tab.g3[f] : L.tab.g3[f]) * (c * c) : 0.0;
        const u64 key = dbits(en);
        const int ex = bits_exp(key);
        const bool hi = v && ex >= whi;
        const bool cp = v && ex < whi && ex >= wlo;
        pe += (v && ex < wlo) ? en : 0.0;
        if (hi && ex == HBINS - 1) slow_bin(gE, en);  // Inf/NaN: counted in the flag bin
        hc += (u32)__popcll(ballot(hi));
        const u64 bc = ballot(cp);
        if (bc) {
          const u32 pos = ncap + (u32)__popcll(bc & ((1ull << lane) - 1ull));
          if (cp) {
            L.key[wv][pos] = key;
            L.idx[wv][pos] = (u32)e;
          }
          ncap += (u32)__popcll(bc);
          if (ncap > (u32)(CAPB - 64)) {
            asm volatile("" ::: "memory");
            cap_flush(L.key[wv], L.idx[wv], ncap, st, list, lidx, j.list_cap, lane);
          }
        }
      }
    }
    hi_tot += hc;
    if (lane == 0) cnt[e] = hc;
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

template <int N, int PREC>
__global__ __launch_bounds__(256, 2) void k_passAL(Job j) {
  __shared__ PassALdsL<N, PREC> L;
  passAL_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L);
}

template <int N, int PREC>
struct PassBLdsL {
  float buf[4][EngL<N, PREC>::LDSW];
  float cst[4][EngL<N, PREC>::n3];  // coefficients by flat index (kept ones are read)
  u64 bm[4][EngL<N, PREC>::W];
  u32 wp[4][EngL<N, PREC>::W];
  TabLdsL<EngL<N, PREC>::n3> tab;
  long long red[4][8];
  __int128 r3[4][3];
  int last;
};

template <int N, int PREC>
DEV void passBL_body(const Job& j, int comp, int vb, int nvb, PassBLdsL<N, PREC>& L, bool tail) {
  typedef EngL<N, PREC> G;
  constexpr int n2 = G::n2, n3 = G::n3, W = G::W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const XParm PR = xparm(st->xm_err, j.xh);
  HistBin* gR = j.histR + (size_t)comp * HBINS;
  const u64 tk = dbits(st->tau);
  u64 voff = 0ull;
  for (int cc = 0; cc < comp; ++cc) voff += j.st[cc].kept;
  const u64 vcap = (u64)j.ncomp * (u64)j.n_elem * (u64)n3;
  const long long E = j.n_elem;
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
  float* cst = L.cst[wv];
  u64* bm = L.bm[wv];
  u32* wp = L.wp[wv];
  for (long long e = (long long)vb * 4 + wv; e < E; e += nw) {
    const double jac = j.jac ? j.jac[e] : 1.0;
    const double* tile = ub + e * n3;
    fwd_l<G>(tile, buf, mt, lane, [](int, double) {});
    for (int k = lane; k < W; k += 64) bm[k] = 0ull;
    asm volatile("" ::: "memory");
    // last forward stage, keep decisions, bitmap, staged values, first
    // inverse stage (in place: this block's positions only)
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float x[4], y[4], cm[4];
      G::template rd<3>(buf, b, x, lane);
      G::mfma(x, y, mt.fa, mt.ha, mt.la);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool v = G::valid(b, m, lane);
        const int f = G::axis(m, lane) * n2 + G::pencil(b, lane);
        const double c = (double)y[m];
        const double en = v ? (j.jac ? jac * L.tab.g3[f] : L.tab.g3[f]) * (c * c) : 0.0;
        const bool keep = v && dbits(en) >= tk;
        cm[m] = keep ? y[m] : 0.0f;
        if (keep) cst[f] = y[m];
        // the 16 lanes of group g hold pencils 16 b .. 16 b + 15 at index 4 g + m
        const u64 bal = ballot(keep);
        if (lane == 0 && bal) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int ax = 4 * g + m;
            const u64 bits = (bal >> (16 * g)) & 0xFFFFull;
            if (ax >= G::n || bits == 0ull) continue;
            const int f0 = ax * n2 + 16 * b, w = f0 >> 6, o = f0 & 63;
            // pencils beyond n2 never keep, so the run stays inside this index
            atomicOr(&bm[w], bits << o);
            if (o > 48 && (bits >> (64 - o)) != 0ull) atomicOr(&bm[w + 1], bits >> (64 - o));
          }
        }
      }
      G::mfma(cm, y, mt.fv, mt.hv, mt.lv);
      G::template wr<3>(buf, b, y, lane);
    }
    asm volatile("" ::: "memory");
    // bitmap out, prefixes, element count check
    u32 run = 0u;
    for (int w0 = 0; w0 < W; w0 += 64) {
      const int w = w0 + lane;
      const u64 wd = w < W ? bm[w] : 0ull;
      if (w < W) gbm[e * W + w] = wd;
      const u32 pc = (u32)__popcll(wd);
      u32 incl = pc;
      for (int d = 1; d < 64; d <<= 1) {
        const u32 o = (u32)__shfl_up((int)incl, d);
        if (lane >= d) incl += o;
      }
      if (w < W) wp[w] = run + incl - pc;
      run += (u32)__shfl((int)incl, 63);
    }
    const u64 ebase = eptr[e];
    if ((u64)run != eptr[e + 1] - ebase) bad = true;
    asm volatile("" ::: "memory");
    // kept values in flat-index order: lane = bit of word w
    for (int w = 0; w < W; ++w) {
      const u64 wd = bm[w];
      if (!((wd >> lane) & 1ull)) continue;
      const u64 pos = voff + ebase + wp[w] + (u64)__popcll(wd & ((1ull << lane) - 1ull));
      if (pos >= vcap) {
        bad = true;
        continue;
      }
      const float val = cst[64 * w + lane];
      if (j.vbytes == 8)
        ((double*)j.values)[pos] = (double)val;
      else
        ((float*)j.values)[pos] = val;
    }
    G::template stage<2>(buf, mt.fv, mt.hv, mt.lv, lane);
    // last inverse stage and the error terms (field values reloaded)
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float x[4], y[4];
      G::template rd<1>(buf, b, x, lane);
      G::mfma(x, y, mt.fv, mt.hv, mt.lv);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool v = G::valid(b, m, lane);
        const int q = G::pencil(b, lane) * G::n + G::axis(m, lane);
        const double u = v ? tile[q] : 0.0;
        const double d = u - (double)y[m];
        const double xv = v ? (j.jac ? jac * L.tab.w3[q] : L.tab.w3[q]) * (d * d) : 0.0;
        pr += xv;
      }
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

template <int N, int PREC>
__global__ __launch_bounds__(256, 2) void k_passBL(Job j) {
  __shared__ PassBLdsL<N, PREC> L;
  passBL_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L, false);
}

// ---- decompress of blobs made by this engine --------------------------------------
// Kept values into pass B's first inverse stage (the same blocks, slots and
// in-place LDS positions), then its remaining stages: the reconstruction pass
// B measured, bit for bit.  One element per wavefront.
template <int N, int PREC>
__global__ __launch_bounds__(256, 2) void k_decompL(Job j, void* out, int out_fp64) {
  typedef EngL<N, PREC> G;
  constexpr int n = G::n, n2 = G::n2, n3 = G::n3, W = G::W;
  __shared__ float bufs[4][G::LDSW];
  __shared__ u64 bms[4][W];
  __shared__ u32 wps[4][W];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  typename G::Mats mt;
  G::init(mt, j.tab, lane);
  float* buf = bufs[wv];
  u64* bm = bms[wv];
  u32* wp = wps[wv];
  const long long E = j.n_elem, total = E * j.ncomp;
  for (long long tk = (long long)blockIdx.x * 4 + wv; tk < total; tk += (long long)gridDim.x * 4) {
    const int comp = (int)(tk / E);
    const long long e = tk % E;
    const u64* gbm = j.bitmap + ((size_t)comp * E + e) * W;
    const u64 base = j.voff[comp] + j.elem_ptr[(size_t)comp * (E + 1) + e];
    for (int w = lane; w < W; w += 64) bm[w] = gbm[w];
    asm volatile("" ::: "memory");
    if (lane == 0) {
      u32 run = 0u;
      for (int w = 0; w < W; ++w) {
        wp[w] = run;
        run += (u32)__popcll(bm[w]);
      }
    }
    asm volatile("" ::: "memory");
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float cm[4], y[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        cm[m] = 0.0f;
        if (!G::valid(b, m, lane)) continue;
        const int f = G::axis(m, lane) * n2 + G::pencil(b, lane), w = f >> 6;
        const u64 wd = bm[w];
        if ((wd >> (f & 63)) & 1ull) {
          const u64 pos = base + wp[w] + (u64)__popcll(wd & ((1ull << (f & 63)) - 1ull));
          cm[m] = j.vbytes == 8 ? (float)((const double*)j.values)[pos] : ((const float*)j.values)[pos];
        }
      }
      G::mfma(cm, y, mt.fv, mt.hv, mt.lv);
      G::template wr<3>(buf, b, y, lane);
    }
    asm volatile("" ::: "memory");
    G::template stage<2>(buf, mt.fv, mt.hv, mt.lv, lane);
    const size_t ob = ((size_t)comp * E + e) * n3;
#pragma unroll 1
    for (int b = 0; b < G::NB; ++b) {
      float x[4], y[4];
      G::template rd<1>(buf, b, x, lane);
      G::mfma(x, y, mt.fv, mt.hv, mt.lv);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (!G::valid(b, m, lane)) continue;
        const size_t o = ob + (size_t)G::pencil(b, lane) * n + G::axis(m, lane);
        if (out_fp64)
          ((double*)out)[o] = (double)y[m];
        else
          ((float*)out)[o] = y[m];
      }
    }
    asm volatile("" ::: "memory");
  }
}

#define ISR_FAST_ORDERS_L(X) X(8) X(9) X(10) X(11)

template <int PREC>
hipError_t launch_decompL_prec(const Job& j, int gx, hipStream_t s, void* out, int out_fp64) {
  switch (j.order) {
#define CASE(NN)                                                                             \
  case NN:                                                                                   \
    hipLaunchKernelGGL((k_decompL<NN, PREC>), dim3(gx), dim3(256), 0, s, j, out, out_fp64); \
    break;
    ISR_FAST_ORDERS_L(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_fast_l(int kind, const Job& j, int gx, hipStream_t s) {
  const dim3 grid(gx, j.ncomp), blk(256);
  switch (j.order) {
#define CASE(NN)                                                    \
  case NN:                                                          \
    if (kind == F_SAMPLE)                                           \
      hipLaunchKernelGGL((k_sampleL<NN, PREC>), grid, blk, 0, s, j); \
    else if (kind == F_PASSA)                                       \
      hipLaunchKernelGGL((k_passAL<NN, PREC>), grid, blk, 0, s, j);  \
    else if (kind == F_PASSB)                                       \
      hipLaunchKernelGGL((k_passBL<NN, PREC>), grid, blk, 0, s, j);  \
    else                                                            \
      return hipErrorInvalidValue;                                  \
    break;
    ISR_FAST_ORDERS_L(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
int resident_fast_l(int kind, int order) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (order) {
#define CASE(NN)                                                                                          \
  case NN:                                                                                                \
    if (kind == F_SAMPLE)                                                                                 \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_sampleL<NN, PREC>, 256, 0);   \
    else if (kind == F_PASSA)                                                                             \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passAL<NN, PREC>, 256, 0);    \
    else if (kind == F_PASSB)                                                                             \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_passBL<NN, PREC>, 256, 0);    \
    break;
    ISR_FAST_ORDERS_L(CASE)
#undef CASE
    default:
      break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace isr
