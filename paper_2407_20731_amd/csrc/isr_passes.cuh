// Streaming passes over the field (templated on the order N and the
// transform precision), shared by isr_pass_fp64.hip / _fp32.hip / _bf16.hip.
//
//   pass1      norm terms + energies -> exact LDS-windowed histograms
//   pass2      energies in the boundary bin -> candidate list
//   pass3      keep e >= tau, bitmaps, decoupled look-back offsets, kept
//              values, inverse transform of the kept set, exact error terms
//   decompress blob -> nodal field (FP64 fixed-order inverse)
//   forward    coefficients only
//
// A workgroup handles EPI elements at a time; the next tile is prefetched into
// registers while the current one is transformed.
#pragma once

#include "isr_common.cuh"

namespace isr {

enum { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// Jacobian-weighted table entry: (J_e * t), J_e = 1 when absent.
DEV double jw(const double* jac, long long e, double t) { return jac ? jac[e] * t : t; }

// ---- register prefetch of one tile (coalesced, 8-byte loads) ---------------
template <int T, int TILE>
struct Prefetch {
  static constexpr int PER = (TILE + T - 1) / T;
  double r[PER];
  DEV void load(const double* __restrict__ src, int count, int tid) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * T;
      r[k] = idx < count ? __builtin_nontemporal_load(&src[idx]) : 0.0;
    }
  }
  DEV void store(double* __restrict__ dst, int count, int tid) const {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * T;
      if (idx < count) dst[idx] = r[k];
    }
  }
};

// ---- FP64 fixed-order transform (VALU, separate multiply and add) ----------
// Every stage uses the thread decomposition el = tid / n2, a = (tid % n2) / n,
// b = tid % n: forward stage 1 contracts i of pencil (k=a, j=b), stage 2
// contracts j of column (k=a, p=b), stage 3 contracts k of column (q=a, p=b)
// and leaves c[r] in registers.  The inverse mirrors it (r, then q, then p).
template <int N>
struct Xf64 {
  typedef Shape<N> S;
  static constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
  typedef double work_t;
  struct Smem {
    double A[n * n];
    double V[n * n];
  };
  struct Regs {};
  static DEV void init(Smem& sm, Regs&, const DevTables& t, int tid, int nthr) {
    for (int k = tid; k < n * n; k += nthr) {
      sm.A[k] = t.A[k];
      sm.V[k] = t.V[k];
    }
  }
  // forward of the tile in `su` (work == su allowed: stages run in place)
  static DEV void forward(const double* su, double* w, const Smem& sm, const Regs&, int el, int a, int b, bool act,
                          int /*ne*/, double (&c)[n]) {
    if (act) {
      const double* pin = su + el * n3 + (a * n + b) * n;
      double x[n], y[n];
#pragma unroll
      for (int i = 0; i < n; ++i) x[i] = pin[i];
      contract64<n>(sm.A, x, y);
      double* pout = w + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) pout[i] = y[i];
    }
    __syncthreads();
    if (act) {
      double* col = w + el * n3 + a * n2 + b;
      double x[n], y[n];
#pragma unroll
      for (int j = 0; j < n; ++j) x[j] = col[j * n];
      contract64<n>(sm.A, x, y);
#pragma unroll
      for (int j = 0; j < n; ++j) col[j * n] = y[j];
    }
    __syncthreads();
    if (act) {
      const double* col = w + el * n3 + a * n + b;
      double x[n];
#pragma unroll
      for (int k = 0; k < n; ++k) x[k] = col[k * n2];
      contract64<n>(sm.A, x, c);
    }
  }
  // inverse of the masked coefficients held by thread (el, q=a, p=b); leaves
  // u~[k=a][j=b][i] in ut
  static DEV void inverse(double* w, const Smem& sm, const Regs&, int el, int a, int b, bool act, int /*ne*/,
                          const double (&cm)[n], double (&ut)[n]) {
    if (act) {
      double y[n];
      contract64<n>(sm.V, cm, y);
      double* col = w + el * n3 + a * n + b;
#pragma unroll
      for (int k = 0; k < n; ++k) col[k * n2] = y[k];
    }
    __syncthreads();
    if (act) {
      double* col = w + el * n3 + a * n2 + b;
      double x[n], y[n];
#pragma unroll
      for (int q = 0; q < n; ++q) x[q] = col[q * n];
      contract64<n>(sm.V, x, y);
#pragma unroll
      for (int j = 0; j < n; ++j) col[j * n] = y[j];
    }
    __syncthreads();
    if (act) {
      const double* pin = w + el * n3 + (a * n + b) * n;
      double x[n];
#pragma unroll
      for (int p = 0; p < n; ++p) x[p] = pin[p];
      contract64<n>(sm.V, x, ut);
    }
  }
};

// ---- MFMA transforms: FP32 (v_mfma_f32_16x16x4_f32) or BF16 split -----------
// One contraction direction at a time, as a GEMM over 16-pencil groups:
// Out[pencil][col] = sum_k X[pencil][k] M[col][k], with the pencils as the
// MFMA rows (A operand), the contracted index k as K (zero padded to the
// instruction's K) and the output index as the 16 columns (B operand = M^T,
// zero padded).  Result lane layout of both instructions: lane l holds rows
// 4*(l/16) + m, m = 0..3, of column l % 16.
//   FP32: X and M rounded to FP32; K = 4 per instruction.
//   BF16: X = Xh + Xl and M = Mh + Ml split into two bf16 each (RNE); three
//         16x16x16 products Xh*Mh + Xh*Ml + Xl*Mh, FP32 accumulation
//         (relative transform error about 2^-16).
DEV short to_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }
DEV float from_bf16(short h) { return __uint_as_float(((u32)(unsigned short)h) << 16); }

// The same split of four values, hi = RN(x) and lo = RN(x - hi), with two
// values per conversion instruction (the pairs land packed, as the MFMA
// operand wants them).
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
DEV u32 pk_bf16(float a, float b) { return __builtin_bit_cast(u32, __builtin_convertvector((fl2){a, b}, bf2)); }
DEV void split_bf16x4(float x0, float x1, float x2, float x3, s4& h, s4& l) {
  const u32 a = pk_bf16(x0, x1), b = pk_bf16(x2, x3);
  const u32 c = pk_bf16(x0 - __uint_as_float(a << 16), x1 - __uint_as_float(a & 0xffff0000u));
  const u32 d = pk_bf16(x2 - __uint_as_float(b << 16), x3 - __uint_as_float(b & 0xffff0000u));
  h = __builtin_bit_cast(s4, (u32x2){a, b});
  l = __builtin_bit_cast(s4, (u32x2){c, d});
}

template <int N, int PREC>
struct XfM {
  typedef Shape<N> S;
  static constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI;
  // K steps of the FP32 instruction: step s, lane group g contracts index
  // 4 g + s (every 16-column engine of the streaming path orders its FP32
  // products this way, so coefficients agree with theirs bit for bit)
  static constexpr int KS = 4;
  static constexpr int GROUPS = (EPI * n2 + 15) / 16;
  static_assert(n <= 16, "one 16-column tile per contraction");
  typedef float work_t;
  struct Smem {};
  struct Frag {
    float f[KS];   // FP32: B operand per K step
    s4 h, l;       // BF16: hi / lo B operand
  };
  struct Regs {
    Frag A, V;
  };
  static DEV void make_frag(Frag& fr, const float* M, int lane) {
    const int col = lane % 16;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * (lane / 16) + s;
      fr.f[s] = (col < n && k < n) ? M[col * n + k] : 0.0f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * (lane / 16) + v;
      const float m = (col < n && k < n) ? M[col * n + k] : 0.0f;
      const short hi = to_bf16(m);
      fr.h[v] = hi;
      fr.l[v] = to_bf16(m - from_bf16(hi));
    }
  }
  static DEV void init(Smem&, Regs& rg, const DevTables& t, int tid, int) {
    const int lane = tid & 63;
    make_frag(rg.A, t.A32, lane);
    make_frag(rg.V, t.V32, lane);
  }
  // One direction over the whole tile: pencil P = (el, a, b) at el*n3 + a*sa +
  // b*sb, contracted index stride si.  In place allowed (src == dst).
  template <class SrcT>
  static DEV void stage(const SrcT* src, float* dst, int sa, int sb, int si, const Frag& fr, int ne, int wave,
                        int nwaves, int lane) {
    for (int g = wave; g < GROUPS; g += nwaves) {
      const int P = g * 16 + (lane % 16);
      const int el = P / n2, rem = P % n2;
      const bool valid = P < EPI * n2 && el < ne;
      const int base = el * n3 + (rem / n) * sa + (rem % n) * sb;
      f4 d = {0.0f, 0.0f, 0.0f, 0.0f};
      if (PREC == P_FP32) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = 4 * (lane / 16) + s;
          const float x = (valid && k < n) ? (float)src[base + k * si] : 0.0f;
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(x, fr.f[s], d, 0, 0, 0);
        }
      } else {
        s4 xh, xl;
        float xv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = 4 * (lane / 16) + v;
          xv[v] = (valid && k < n) ? (float)src[base + k * si] : 0.0f;
        }
        split_bf16x4(xv[0], xv[1], xv[2], xv[3], xh, xl);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xh, fr.h, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xh, fr.l, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xl, fr.h, d, 0, 0, 0);
      }
      const int col = lane % 16;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int P2 = g * 16 + 4 * (lane / 16) + m;
        const int el2 = P2 / n2, rem2 = P2 % n2;
        if (col < n && P2 < EPI * n2 && el2 < ne) dst[el2 * n3 + (rem2 / n) * sa + (rem2 % n) * sb + col * si] = d[m];
      }
    }
  }
  static DEV void forward(const double* su, float* w, const Smem&, const Regs& rg, int el, int a, int b, bool act,
                          int ne, double (&c)[n]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    stage<double>(su, w, n2, n, 1, rg.A, ne, wave, nw, lane);  // i -> p, pencils (k, j)
    __syncthreads();
    stage<float>(w, w, n2, 1, n, rg.A, ne, wave, nw, lane);    // j -> q, pencils (k, p)
    __syncthreads();
    stage<float>(w, w, n, 1, n2, rg.A, ne, wave, nw, lane);    // k -> r, pencils (q, p)
    __syncthreads();
    if (act) {
      const float* col = w + el * n3 + a * n + b;
#pragma unroll
      for (int r = 0; r < n; ++r) c[r] = (double)col[r * n2];
    }
  }
  static DEV void inverse(float* w, const Smem&, const Regs& rg, int el, int a, int b, bool act, int ne,
                          const double (&cm)[n], double (&ut)[n]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (act) {
      float* col = w + el * n3 + a * n + b;
#pragma unroll
      for (int r = 0; r < n; ++r) col[r * n2] = (float)cm[r];
    }
    __syncthreads();
    stage<float>(w, w, n, 1, n2, rg.V, ne, wave, nw, lane);    // r -> k, pencils (q, p)
    __syncthreads();
    stage<float>(w, w, n2, 1, n, rg.V, ne, wave, nw, lane);    // q -> j, pencils (k, p)
    __syncthreads();
    stage<float>(w, w, n2, n, 1, rg.V, ne, wave, nw, lane);    // p -> i, pencils (k, j)
    __syncthreads();
    if (act) {
      const float* pin = w + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) ut[i] = (double)pin[i];
    }
  }
};

template <int N, int PREC>
struct XfSel {
  typedef XfM<N, PREC> type;
};
template <int N>
struct XfSel<N, P_FP64> {
  typedef Xf64<N> type;
};

// ---- grid-level helpers -------------------------------------------------------
DEV void comp_voff(const Job& j, int comp, u64& voff) {
  voff = 0;
  for (int cc = 0; cc < comp; ++cc) voff += j.st[cc].kept;
}

// ---- pass 1 -----------------------------------------------------------------
// sample = 1: only every j.sample_stride-th tile, into the sample histograms
// (predicts the boundary bin).  sample = 0: every tile, into the histograms,
// and energies whose exponent lies in the predicted window [win_lo, win_hi]
// are copied to candidate list 0 (staged in LDS, reserved in bulk).
constexpr int CBUF = 4096;

DEV void cbuf_flush(u64* cbuf, u32* ncb, u64* gbase_s, u64* list, u64* gcount, u64 cap, int* flag, int tid,
                    int nthr) {
  __syncthreads();
  const u32 k = *ncb;
  if (k) {
    if (tid == 0) *gbase_s = atomicAdd(gcount, (u64)k);
    __syncthreads();
    const u64 base = *gbase_s;
    for (u32 i = tid; i < k; i += nthr) {
      if (base + i < cap)
        list[base + i] = cbuf[i];
      else
        atomicOr(flag, ST_LIST);
    }
  }
  __syncthreads();
  if (tid == 0) *ncb = 0u;
  __syncthreads();
}

// wave-aggregated append of key to the LDS candidate buffer
DEV void cbuf_put(u64* cbuf, u32* ncb, bool m, u64 key) {
  const u64 bal = ballot(m);
  if (bal) {
    const int leader = __ffsll((long long)bal) - 1;
    u32 base = 0;
    if (lane_id() == leader) base = atomicAdd(ncb, (u32)__popcll(bal));
    base = (u32)__shfl((int)base, leader);
    if (m) cbuf[base + (u32)__popcll(bal & ((1ull << lane_id()) - 1ull))] = key;
  }
}

template <int N, int PREC>
struct Pass1Lds {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  static constexpr int CB1 = 768;  // flushed whenever fewer than 256 slots (one row of appends) remain
  double su[S::TILE];
  typename X::work_t sw_buf[PREC == P_FP64 ? 1 : S::TILE];
  LdsHist hN, hE;
  typename X::Smem sm;
  u64 cbuf[CB1];
  u32 ncb;
  u64 gbase_s;
};

// Tiles t0, t0 + tstride, ... of component comp.
template <int N, int PREC>
DEV void pass1_body(const Job& j, int comp, long long t0, long long tstride, int sample, Pass1Lds<N, PREC>& L) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  constexpr bool INPLACE = PREC == P_FP64;
  constexpr int CB1 = Pass1Lds<N, PREC>::CB1;
  typename X::Regs rg;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const double* u = j.u + (size_t)comp * j.comp_stride;
  CompState* st = j.st + comp;
  HistBin* gN = (sample ? j.histNs : j.histN) + (size_t)comp * HBINS;
  HistBin* gE = (sample ? j.histEs : j.histE) + (size_t)comp * HBINS;
  const int wlo = sample ? 0 : st->win_lo, whi = sample ? 0 : st->win_hi;  // [wlo, whi)
  const bool capture = wlo < whi;
  u64* list = list_ptr(j, comp, 0);
  typename X::work_t* sw = INPLACE ? (typename X::work_t*)L.su : L.sw_buf;
  __syncthreads();
  lh_init(L.hN, tid, T);
  lh_init(L.hE, tid, T);
  X::init(L.sm, rg, j.tab, tid, T);
  if (tid == 0) L.ncb = 0u;
  Prefetch<T, S::TILE> pf;
  long long t = t0;
  if (t < tiles) {
    const long long e0 = t * EPI;
    pf.load(u + e0 * n3, (int)((E - e0) < EPI ? (E - e0) : EPI) * n3, tid);
  }
  bool first = true;
  for (; t < tiles; t += tstride) {
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    __syncthreads();
    pf.store(L.su, ne * n3, tid);
    __syncthreads();
    const long long tn = t + tstride;
    if (tn < tiles) {
      const long long e1 = tn * EPI;
      pf.load(u + e1 * n3, (int)((E - e1) < EPI ? (E - e1) : EPI) * n3, tid);
    }
    const bool act = tid < S::ACT && el < ne;
    const long long e = e0 + el;
    // norm terms (J_e * w3[k][j][i]) * (u*u) of pencil (k=a, j=b)
    double nt[n];
    if (act) {
      const double* pin = L.su + el * n3 + (a * n + b) * n;
      const double* w3 = j.tab.w3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) nt[i] = jw(j.jac, e, w3[i]) * (pin[i] * pin[i]);
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int i = 0; i < n; ++i) lh_note_max(L.hN, nt[i]);
      }
      __syncthreads();
      if (tid == 0) lh_place(L.hN);
      __syncthreads();
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < n; ++i) lh_insert(L.hN, gN, nt[i]);
    }
    __syncthreads();
    double c[n], en[n];
    X::forward(L.su, sw, L.sm, rg, el, a, b, act, ne, c);
    if (act) {
#pragma unroll
      for (int r = 0; r < n; ++r) en[r] = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int r = 0; r < n; ++r) lh_note_max(L.hE, en[r]);
      }
      __syncthreads();
      if (tid == 0) lh_place(L.hE);
      __syncthreads();
      first = false;
    }
    if (act) {
#pragma unroll
      for (int r = 0; r < n; ++r) lh_insert(L.hE, gE, en[r]);
    }
    if (capture) {
      static_assert(T <= 256, "one row of appends adds at most 256 keys");
#pragma unroll
      for (int r = 0; r < n; ++r) {
        const u64 key = act ? dbits(en[r]) : 0ull;
        const int ex = bits_exp(key);
        cbuf_put(L.cbuf, &L.ncb, act && ex >= wlo && ex < whi, key);
        __syncthreads();
        const bool full = L.ncb > (u32)(CB1 - 256);
        // every thread has read the fill level before the next row appends
        // (else waves could disagree on the flush and meet at different barriers)
        __syncthreads();
        if (full) cbuf_flush(L.cbuf, &L.ncb, &L.gbase_s, list, &st->list_count[0], j.list_cap, &st->flags, tid, T);
      }
    }
  }
  __syncthreads();
  lh_flush(L.hN, gN, tid, T);
  lh_flush(L.hE, gE, tid, T);
  if (capture) cbuf_flush(L.cbuf, &L.ncb, &L.gbase_s, list, &st->list_count[0], j.list_cap, &st->flags, tid, T);
  __syncthreads();
}

template <int N, int PREC>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass1(Job j, int sample) {
  __shared__ Pass1Lds<N, PREC> L;
  const long long tstep = sample ? j.sample_stride : 1;
  pass1_body<N, PREC>(j, blockIdx.y, (long long)blockIdx.x * tstep, (long long)gridDim.x * tstep, sample, L);
}

// ---- pass 2 (only when the boundary bin fell outside the captured window) ----
template <int N, int PREC>
struct Pass2Lds {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  double su[S::TILE];
  typename X::work_t sw_buf[PREC == P_FP64 ? 1 : S::TILE];
  typename X::Smem sm;
  u64 cbuf[CBUF];
  u32 ncb;
  u64 gbase_s;
};

template <int N, int PREC>
DEV void pass2_body(const Job& j, int comp, long long t0, long long tstride, Pass2Lds<N, PREC>& L) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  constexpr bool INPLACE = PREC == P_FP64;
  static_assert(S::TILE <= CBUF, "a whole tile must fit the candidate buffer");
  typename X::Regs rg;
  const int tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->resolved || !st->need_pass2) return;
  const u64 prefix = st->key_prefix, mask = st->key_mask;
  u64* list = list_ptr(j, comp, 0);
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const double* u = j.u + (size_t)comp * j.comp_stride;
  typename X::work_t* sw = INPLACE ? (typename X::work_t*)L.su : L.sw_buf;
  __syncthreads();
  X::init(L.sm, rg, j.tab, tid, T);
  if (tid == 0) L.ncb = 0u;
  Prefetch<T, S::TILE> pf;
  long long t = t0;
  if (t < tiles) {
    const long long e0 = t * EPI;
    pf.load(u + e0 * n3, (int)((E - e0) < EPI ? (E - e0) : EPI) * n3, tid);
  }
  for (; t < tiles; t += tstride) {
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    __syncthreads();
    pf.store(L.su, ne * n3, tid);
    __syncthreads();
    const long long tn = t + tstride;
    if (tn < tiles) {
      const long long e1 = tn * EPI;
      pf.load(u + e1 * n3, (int)((E - e1) < EPI ? (E - e1) : EPI) * n3, tid);
    }
    const bool act = tid < S::ACT && el < ne;
    const long long e = e0 + el;
    double c[n];
    X::forward(L.su, sw, L.sm, rg, el, a, b, act, ne, c);
#pragma unroll
    for (int r = 0; r < n; ++r) {
      u64 key = 0;
      bool m = false;
      if (act) {
        const double en = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
        key = dbits(en);
        m = (key & mask) == prefix;
      }
      cbuf_put(L.cbuf, &L.ncb, m, key);
    }
    __syncthreads();
    if (L.ncb > (u32)(CBUF - S::TILE))
      cbuf_flush(L.cbuf, &L.ncb, &L.gbase_s, list, &st->list_count[0], j.list_cap, &st->flags, tid, T);
  }
  cbuf_flush(L.cbuf, &L.ncb, &L.gbase_s, list, &st->list_count[0], j.list_cap, &st->flags, tid, T);
}

template <int N, int PREC>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass2(Job j) {
  __shared__ Pass2Lds<N, PREC> L;
  pass2_body<N, PREC>(j, blockIdx.y, blockIdx.x, gridDim.x, L);
}

// ---- pass 3 -----------------------------------------------------------------
template <int N, int PREC>
struct Pass3Lds {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  double su[S::TILE];
  typename X::work_t sw[S::TILE];
  typename X::Smem sm;
  LdsHist hR;
  u64 bm[S::EPI * S::W];
  u32 cntl[S::EPI];
  u64 excl_s;
  long long ticket_s;
};

// One tile t of component comp.  The error histogram window in L.hR belongs
// to comp and is flushed by the caller; `first` places it.
template <int N, int PREC>
DEV void pass3_tile(const Job& j, int comp, long long t, Pass3Lds<N, PREC>& L,
                    const typename XfSel<N, PREC>::type::Regs& rg, bool& first) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS, W = S::W;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const double tau_c = j.st[comp].tau;
  const long long e0 = t * EPI;
  const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
  const double* u = j.u + (size_t)comp * j.comp_stride;
  {
    Prefetch<T, S::TILE> pf;
    pf.load(u + e0 * n3, ne * n3, tid);
    pf.store(L.su, ne * n3, tid);
  }
  for (int k = tid; k < EPI * W; k += T) L.bm[k] = 0ull;
  __syncthreads();
  const bool act = tid < S::ACT && el < ne;
  const long long e = e0 + el;
  double c[n];
  bool keep[n];
  X::forward(L.su, L.sw, L.sm, rg, el, a, b, act, ne, c);
  if (act) {
    const double tau = j.tau_elem ? j.tau_elem[(size_t)comp * E + e] : tau_c;
#pragma unroll
    for (int r = 0; r < n; ++r) {
      const double en = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
      keep[r] = en >= tau;
      if (keep[r]) {
        const int f = (r * n + a) * n + b;
        atomicOr(&L.bm[el * W + (f >> 6)], 1ull << (f & 63));
      }
    }
  }
  __syncthreads();
  if (tid < EPI) {
    u32 s = 0;
    if (tid < ne)
      for (int w = 0; w < W; ++w) s += (u32)__popcll(L.bm[tid * W + w]);
    L.cntl[tid] = s;
  }
  __syncthreads();
  u64* lb = j.lookback + (size_t)comp * tiles;
  // publish the aggregate and resolve the prefix at once, so that inclusive
  // prefixes follow closely behind the tiles being claimed and look-backs
  // stay short
  if (tid < 64) {
    lookback_publish(lb, t, L.cntl, ne, &L.excl_s);
    lookback_wait(lb, t, L.cntl, ne, &j.st[comp].flags, &L.excl_s);
  }
  double et[n];
  {
    double cm[n], ut[n];
#pragma unroll
    for (int r = 0; r < n; ++r) cm[r] = (act && keep[r]) ? c[r] : 0.0;
    X::inverse(L.sw, L.sm, rg, el, a, b, act, ne, cm, ut);
    if (act) {
      const double* w3 = j.tab.w3 + (a * n + b) * n;
      const double* pu = L.su + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double d = pu[i] - ut[i];
        et[i] = jw(j.jac, e, w3[i]) * (d * d);
      }
    }
  }
  if (first) {
    if (act) {
#pragma unroll
      for (int i = 0; i < n; ++i) lh_note_max(L.hR, et[i]);
    }
    __syncthreads();
    if (tid == 0) lh_place(L.hR);
    __syncthreads();
    first = false;
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < n; ++i) lh_insert(L.hR, j.histR + (size_t)comp * HBINS, et[i]);
  }
  __syncthreads();
  const u64 ex = L.excl_s;
  u64* gbm = j.bitmap + ((size_t)comp * E + e0) * W;
  for (int k = tid; k < ne * W; k += T) gbm[k] = L.bm[k];
  u64* gptr = j.elem_ptr + (size_t)comp * (E + 1);
  if (tid < ne) {
    u64 o = ex;
    for (int k = 0; k < tid; ++k) o += L.cntl[k];
    gptr[e0 + tid] = o;
    if (e0 + tid == E - 1) gptr[E] = o + L.cntl[tid];
  }
  if (act) {
    u64 voff;
    comp_voff(j, comp, voff);
    u64 eoff = ex;
    for (int k = 0; k < el; ++k) eoff += L.cntl[k];
#pragma unroll
    for (int r = 0; r < n; ++r) {
      if (!keep[r]) continue;
      const int f = (r * n + a) * n + b;
      const int wi = f >> 6;
      u32 rank = 0;
      for (int w = 0; w < wi; ++w) rank += (u32)__popcll(L.bm[el * W + w]);
      rank += (u32)__popcll(L.bm[el * W + wi] & ((1ull << (f & 63)) - 1ull));
      const u64 pos = voff + eoff + rank;
      if (j.vbytes == 8)
        ((double*)j.values)[pos] = c[r];
      else
        ((float*)j.values)[pos] = (float)c[r];
    }
  }
  __syncthreads();
}

template <int N, int PREC>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass3(Job j) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int EPI = S::EPI, T = S::THREADS;
  __shared__ Pass3Lds<N, PREC> L;
  typename X::Regs rg;
  const int tid = threadIdx.x;
  const long long tiles = (j.n_elem + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
  lh_init(L.hR, tid, T);
  X::init(L.sm, rg, j.tab, tid, T);
  int cur = -1;
  bool first = true;
  for (;;) {
    __syncthreads();
    if (tid == 0) L.ticket_s = (long long)atomicAdd(&j.ticket[0], 1u);
    __syncthreads();
    const long long tk = L.ticket_s;
    if (tk >= total) break;
    const int comp = (int)(tk / tiles);
    if (comp != cur) {
      if (cur >= 0) {
        lh_flush(L.hR, j.histR + (size_t)cur * HBINS, tid, T);
        __syncthreads();
        lh_init(L.hR, tid, T);
        __syncthreads();
      }
      cur = comp;
      first = true;
    }
    pass3_tile<N, PREC>(j, comp, tk % tiles, L, rg, first);
  }
  __syncthreads();
  if (cur >= 0) lh_flush(L.hR, j.histR + (size_t)cur * HBINS, tid, T);
}

// ---- decompress ------------------------------------------------------------------
// The inverse of the blob's kept values with the transform of its precision:
// FP64 blobs with the fixed-order FP64 inverse (the oracle's); FP32 / BF16
// blobs compressed on these general passes with the same MFMA inverse as
// pass 3, so that the reconstruction is the one whose error the compression
// measured, bit for bit (each pencil's result depends only on its own
// values, not on the tile it shares an instruction with).
template <int N, int PREC>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_decompress(Job j, void* out, int out_fp64) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS, W = S::W;
  __shared__ typename X::work_t sw[S::TILE];
  __shared__ typename X::Smem sm;
  __shared__ u64 bm[EPI * W];
  typename X::Regs rg;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
  X::init(sm, rg, j.tab, tid, T);
  for (long long tk = blockIdx.x; tk < total; tk += gridDim.x) {
    const int comp = (int)(tk / tiles);
    const long long t = tk % tiles;
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    const u64* gbm = j.bitmap + ((size_t)comp * E + e0) * W;
    __syncthreads();
    for (int k = tid; k < EPI * W; k += T) bm[k] = k < ne * W ? gbm[k] : 0ull;
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    const u64 voff = j.voff[comp];
    double cm[n], ut[n];
#pragma unroll
    for (int r = 0; r < n; ++r) cm[r] = 0.0;
    if (act) {
      const u64 base = voff + j.elem_ptr[(size_t)comp * (E + 1) + e0 + el];
#pragma unroll
      for (int r = 0; r < n; ++r) {
        const int f = (r * n + a) * n + b;
        const int wi = f >> 6;
        const u64 word = bm[el * W + wi];
        if ((word >> (f & 63)) & 1ull) {
          u32 rank = 0;
          for (int w = 0; w < wi; ++w) rank += (u32)__popcll(bm[el * W + w]);
          rank += (u32)__popcll(word & ((1ull << (f & 63)) - 1ull));
          cm[r] = j.vbytes == 8 ? ((const double*)j.values)[base + rank]
                                : (double)((const float*)j.values)[base + rank];
          // quantisation codes: the value is (code * step) / sqrt(g3)
          if (j.qstep) cm[r] = (cm[r] * j.qstep[comp]) / __builtin_sqrt(j.tab.g3[f]);
        }
      }
    }
    X::inverse(sw, sm, rg, el, a, b, act, ne, cm, ut);
    if (act) {
      const size_t o = ((size_t)comp * E + e0 + el) * n3 + (size_t)(a * n + b) * n;
      if (out_fp64) {
#pragma unroll
        for (int i = 0; i < n; ++i) ((double*)out)[o + i] = ut[i];
      } else {
#pragma unroll
        for (int i = 0; i < n; ++i) ((float*)out)[o + i] = (float)ut[i];
      }
    }
  }
}

// ---- quantised variant: codes of the kept values and the error they leave ------
// Per tile: every kept FP64 coefficient c of the blob gets the code
// q = rint((c sqrt(g3)) / step), written as an FP32 integer at the value's
// position; the dequantised (q step) / sqrt(g3) go through the fixed-order
// FP64 inverse (the one decompression uses), and the terms w3 (u - u~)^2 into
// the exact error histogram j.histR.  A code of magnitude 2^24 or more sets
// j.ticket[1].  Unit Jacobians.
template <int N>
struct QuantLds {
  typedef Shape<N> S;
  double su[S::TILE];
  double sw[S::TILE];
  typename Xf64<N>::Smem sm;
  LdsHist hR;
  u64 bm[S::EPI * S::W];
};

template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_quantize(Job j) {
  typedef Shape<N> S;
  typedef Xf64<N> X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS, W = S::W;
  __shared__ QuantLds<N> L;
  typename X::Regs rg;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem, tiles = (E + EPI - 1) / EPI, total = tiles * j.ncomp;
  lh_init(L.hR, tid, T);
  X::init(L.sm, rg, j.tab, tid, T);
  int cur = -1;
  bool first = true;
  for (long long tk = blockIdx.x; tk < total; tk += gridDim.x) {
    const int comp = (int)(tk / tiles);
    if (comp != cur) {
      if (cur >= 0) {
        __syncthreads();
        lh_flush(L.hR, j.histR + (size_t)cur * HBINS, tid, T);
        __syncthreads();
        lh_init(L.hR, tid, T);
      }
      cur = comp;
      first = true;
    }
    const long long e0 = (tk % tiles) * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    __syncthreads();
    {
      Prefetch<T, S::TILE> pf;
      pf.load(j.u + (size_t)comp * j.comp_stride + e0 * n3, ne * n3, tid);
      pf.store(L.su, ne * n3, tid);
    }
    const u64* gbm = j.bitmap + ((size_t)comp * E + e0) * W;
    for (int k = tid; k < EPI * W; k += T) L.bm[k] = k < ne * W ? gbm[k] : 0ull;
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    const double step = j.qstep[comp];
    double cm[n], ut[n];
#pragma unroll
    for (int r = 0; r < n; ++r) cm[r] = 0.0;
    if (act) {
      const u64 base = j.voff[comp] + j.elem_ptr[(size_t)comp * (E + 1) + e0 + el];
#pragma unroll
      for (int r = 0; r < n; ++r) {
        const int f = (r * n + a) * n + b;
        const int wi = f >> 6;
        const u64 word = L.bm[el * W + wi];
        if ((word >> (f & 63)) & 1ull) {
          u32 rank = 0;
          for (int w = 0; w < wi; ++w) rank += (u32)__popcll(L.bm[el * W + w]);
          rank += (u32)__popcll(word & ((1ull << (f & 63)) - 1ull));
          const double c = ((const double*)j.values)[base + rank];
          const double sq = __builtin_sqrt(j.tab.g3[f]);
          const double q = __builtin_rint((c * sq) / step);
          if (!(__builtin_fabs(q) < 16777216.0)) atomicOr(&j.ticket[1], 1u);
          j.qvals[base + rank] = (float)q;
          cm[r] = (q * step) / sq;
        }
      }
    }
    X::inverse(L.sw, L.sm, rg, el, a, b, act, ne, cm, ut);
    double et[n];
    if (act) {
      const double* w3 = j.tab.w3 + (a * n + b) * n;
      const double* pu = L.su + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double d = pu[i] - ut[i];
        et[i] = w3[i] * (d * d);
      }
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int i = 0; i < n; ++i) lh_note_max(L.hR, et[i]);
      }
      __syncthreads();
      if (tid == 0) lh_place(L.hR);
      __syncthreads();
      first = false;
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < n; ++i) lh_insert(L.hR, j.histR + (size_t)comp * HBINS, et[i]);
    }
  }
  __syncthreads();
  if (cur >= 0) lh_flush(L.hR, j.histR + (size_t)cur * HBINS, tid, T);
}

// ---- forward transform only -----------------------------------------------------
template <int N, int PREC>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_forward(Job j, void* coef) {
  typedef Shape<N> S;
  typedef typename XfSel<N, PREC>::type X;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  constexpr bool INPLACE = PREC == P_FP64;
  __shared__ double su[S::TILE];
  __shared__ typename X::work_t sw_buf[INPLACE ? 1 : S::TILE];
  __shared__ typename X::Smem sm;
  typename X::Regs rg;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
  typename X::work_t* sw = INPLACE ? (typename X::work_t*)su : sw_buf;
  X::init(sm, rg, j.tab, tid, T);
  for (long long tk = blockIdx.x; tk < total; tk += gridDim.x) {
    const int comp = (int)(tk / tiles);
    const long long t = tk % tiles;
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    __syncthreads();
    {
      Prefetch<T, S::TILE> pf;
      pf.load(j.u + (size_t)comp * j.comp_stride + e0 * n3, ne * n3, tid);
      pf.store(su, ne * n3, tid);
    }
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    double c[n];
    X::forward(su, sw, sm, rg, el, a, b, act, ne, c);
    __syncthreads();
    if (act) {
      double* col = su + el * n3 + a * n + b;
#pragma unroll
      for (int r = 0; r < n; ++r) col[r * n2] = c[r];
    }
    __syncthreads();
    const size_t obase = ((size_t)comp * E + e0) * n3;
    if (PREC == P_FP64) {
      double* o = (double*)coef + obase;
      for (int k = tid; k < ne * n3; k += T) o[k] = su[k];
    } else {
      float* o = (float*)coef + obase;
      for (int k = tid; k < ne * n3; k += T) o[k] = (float)su[k];
    }
  }
}

// ---- launchers for one precision ----------------------------------------------
#define ISR_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

template <int PREC>
hipError_t launch_pass_prec(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i) {
  switch (j.order) {
#define CASE(NN)                                                                                                  \
  case NN: {                                                                                                      \
    const dim3 blk(Shape<NN>::THREADS);                                                                           \
    if (kind == K_PASS1)                                                                                          \
      hipLaunchKernelGGL((k_pass1<NN, PREC>), dim3(grid, j.ncomp), blk, 0, s, j, extra_i);                        \
    else if (kind == K_PASS2)                                                                                     \
      hipLaunchKernelGGL((k_pass2<NN, PREC>), dim3(grid, j.ncomp), blk, 0, s, j);                                 \
    else if (kind == K_PASS3)                                                                                     \
      hipLaunchKernelGGL((k_pass3<NN, PREC>), dim3(grid), blk, 0, s, j);                                          \
    else if (kind == K_FORWARD)                                                                                   \
      hipLaunchKernelGGL((k_forward<NN, PREC>), dim3(grid), blk, 0, s, j, extra);                                 \
    else if (kind == K_DECOMP)                                                                                    \
      hipLaunchKernelGGL((k_decompress<NN, PREC>), dim3(grid), blk, 0, s, j, extra, extra_i);                     \
    else if (kind == K_QUANT && PREC == P_FP64)                                                                   \
      hipLaunchKernelGGL((k_quantize<NN>), dim3(grid), blk, 0, s, j);                                             \
    else                                                                                                          \
      return hipErrorInvalidValue;                                                                                \
    break;                                                                                                        \
  }
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
int resident_prec(int kind, int order) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (order) {
#define CASE(NN)                                                                                                  \
  case NN: {                                                                                                      \
    const int blk = Shape<NN>::THREADS;                                                                           \
    if (kind == K_PASS1)                                                                                          \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pass1<NN, PREC>, blk, 0);             \
    else if (kind == K_PASS2)                                                                                     \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pass2<NN, PREC>, blk, 0);             \
    else if (kind == K_PASS3)                                                                                     \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pass3<NN, PREC>, blk, 0);             \
    else if (kind == K_FORWARD)                                                                                   \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_forward<NN, PREC>, blk, 0);           \
    break;                                                                                                        \
  }
    ISR_ORDERS(CASE)
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
