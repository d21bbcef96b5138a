// HIP kernels for gfx950 (CDNA4): in-situ reduction of spectral-element
// snapshots (arXiv 2407.20731, Sec. IV-B), FP64 fixed-order path.
//
// Phases per snapshot (one kernel each, all on the caller's stream):
//   pass1     read the field once: per-element forward transform, exact
//             histograms of the mass-weighted norm terms and of the energies
//   select1   norm U2 (exact), budget B, boundary exponent bin of tau
//   pass2     read the field again: energies in the boundary bin -> list
//   refine    levels 2..6: histogram of the next fraction bits of the listed
//   select    energies, then pick the sub-bin that holds tau (or sort a
//             small sub-bin and resolve tau exactly)
//   pass3     read the field a third time: recompute coefficients, keep
//             e >= tau, wave-ballot bitmaps, decoupled look-back scan of the
//             kept counts, compacted values, inverse transform, exact error
//   finalize  err2, rel, dropped energy
#include "isr_common.cuh"

namespace isr {

// --------------------------------------------------------------------------
// small utilities

__global__ void k_zero(u64* p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0ull;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t nw = bytes / 8;
  if (nw == 0) return hipSuccess;
  int grid = (int)((nw + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, (u64*)p, nw);
  return hipGetLastError();
}

// Jacobian-weighted table entry: (J_e * t) with J_e == 1 when absent.
DEV double jw(const double* jac, long long e, double t) { return jac ? jac[e] * t : t; }

// --------------------------------------------------------------------------
// forward transform of one tile held in LDS (in place), FP64 fixed order.
// Thread decomposition for every stage: el = tid / n2, a = (tid % n2) / n,
// b = tid % n.  Stage 1 contracts i for pencil (k=a, j=b); stage 2 contracts
// j for column (k=a, p=b); stage 3 contracts k for column (q=a, p=b) and
// leaves c[r][q][p], r = 0..n-1, in registers.

template <int N>
struct Fwd64 {
  typedef Shape<N> S;
  static constexpr int n = S::n, n2 = S::n2, n3 = S::n3;

  // stage 1: x <- pencil, t1 <- A x written to dst pencil
  static DEV void stage1(const double* __restrict__ src, double* __restrict__ dst,
                         const double* __restrict__ A, int el, int a, int b, double (&x)[n]) {
    const double* pin = src + el * n3 + (a * n + b) * n;
#pragma unroll
    for (int i = 0; i < n; ++i) x[i] = pin[i];
    double y[n];
    contract64<n>(A, x, y);
    double* pout = dst + el * n3 + (a * n + b) * n;
#pragma unroll
    for (int i = 0; i < n; ++i) pout[i] = y[i];
  }
  // stage 2: column (k=a, p=b) along j, in place
  static DEV void stage2(double* __restrict__ buf, const double* __restrict__ A, int el, int a, int b) {
    double* col = buf + el * n3 + a * n2 + b;
    double x[n], y[n];
#pragma unroll
    for (int j = 0; j < n; ++j) x[j] = col[j * n];
    contract64<n>(A, x, y);
#pragma unroll
    for (int j = 0; j < n; ++j) col[j * n] = y[j];
  }
  // stage 3: column (q=a, p=b) along k, result in registers
  static DEV void stage3(const double* __restrict__ buf, const double* __restrict__ A, int el, int a, int b,
                         double (&c)[n]) {
    const double* col = buf + el * n3 + a * n + b;
    double x[n];
#pragma unroll
    for (int k = 0; k < n; ++k) x[k] = col[k * n2];
    contract64<n>(A, x, c);
  }
};

// inverse transform (fixed order: r, then q, then p) of coefficients held in
// registers by thread (el, q=a, p=b); the final stage leaves u~[k=a][j=b][i]
// in registers of thread (el, a, b).
template <int N>
struct Inv64 {
  typedef Shape<N> S;
  static constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
  // stage A: column (q=a, p=b): s1[k] = sum_r V[k][r] c[r], written to buf
  static DEV void stageA(double* __restrict__ buf, const double* __restrict__ V, int el, int a, int b,
                         const double (&c)[n]) {
    double y[n];
    contract64<n>(V, c, y);
    double* col = buf + el * n3 + a * n + b;
#pragma unroll
    for (int k = 0; k < n; ++k) col[k * n2] = y[k];
  }
  // stage B: column (k=a, p=b) along q -> j, in place
  static DEV void stageB(double* __restrict__ buf, const double* __restrict__ V, int el, int a, int b) {
    double* col = buf + el * n3 + a * n2 + b;
    double x[n], y[n];
#pragma unroll
    for (int q = 0; q < n; ++q) x[q] = col[q * n];
    contract64<n>(V, x, y);
#pragma unroll
    for (int j = 0; j < n; ++j) col[j * n] = y[j];
  }
  // stage C: pencil (k=a, j=b) along p -> i, result in registers
  static DEV void stageC(const double* __restrict__ buf, const double* __restrict__ V, int el, int a, int b,
                         double (&u)[n]) {
    const double* pin = buf + el * n3 + (a * n + b) * n;
    double x[n];
#pragma unroll
    for (int p = 0; p < n; ++p) x[p] = pin[p];
    contract64<n>(V, x, u);
  }
};

// --------------------------------------------------------------------------
// pass 1: norm terms and energies into exact histograms.
// grid = (gx, ncomp); each workgroup walks tiles of its component.

template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass1(Job j) {
  typedef Shape<N> S;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  __shared__ double tile[S::TILE];
  __shared__ LdsHist hN, hE;
  const int tid = threadIdx.x, comp = blockIdx.y;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const double* u = j.u + (size_t)comp * j.comp_stride;
  HistBin* gN = j.histN + (size_t)comp * HBINS;
  HistBin* gE = j.histE + (size_t)comp * HBINS;
  lh_init(hN, tid, T);
  lh_init(hE, tid, T);
  __syncthreads();
  bool first = true;
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    load_tile<T>(tile, u + e0 * n3, ne * n3, tid);
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    const long long e = e0 + el;
    // stage 1 + norm terms (J_e * w3[k][j][i]) * (u*u)
    double x[n], nt[n];
    if (act) {
      Fwd64<N>::stage1(tile, tile, j.tab.A, el, a, b, x);
      const double* w3 = j.tab.w3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) nt[i] = jw(j.jac, e, w3[i]) * (x[i] * x[i]);
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int i = 0; i < n; ++i) lh_note_max(hN, nt[i]);
      }
      __syncthreads();
      if (tid == 0) lh_place(hN);
      __syncthreads();
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < n; ++i) lh_insert(hN, gN, nt[i]);
    }
    __syncthreads();
    if (act) Fwd64<N>::stage2(tile, j.tab.A, el, a, b);
    __syncthreads();
    double c[n], en[n];
    if (act) {
      Fwd64<N>::stage3(tile, j.tab.A, el, a, b, c);
#pragma unroll
      for (int r = 0; r < n; ++r) en[r] = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int r = 0; r < n; ++r) lh_note_max(hE, en[r]);
      }
      __syncthreads();
      if (tid == 0) lh_place(hE);
      __syncthreads();
      first = false;
    }
    if (act) {
#pragma unroll
      for (int r = 0; r < n; ++r) lh_insert(hE, gE, en[r]);
    }
    __syncthreads();
  }
  lh_flush(hN, gN, tid, T);
  lh_flush(hE, gE, tid, T);
}

// --------------------------------------------------------------------------
// select, level 1 (one wave per component): U2, B, the slack integer
// Tint = largest X-unit sum whose round-to-nearest is <= B, and the boundary
// exponent bin b*: the last non-empty bin whose exclusive prefix sum is <= Tint.

__global__ __launch_bounds__(64) void k_select1(Job j) {
  const int comp = blockIdx.x, lane = threadIdx.x;
  CompState* st = j.st + comp;
  const HistBin* HN = j.histN + (size_t)comp * HBINS;
  const HistBin* HE = j.histE + (size_t)comp * HBINS;
  const double tol = j.tol;
  int flags = 0;
  if (HN[HBINS - 1].cnt) flags |= ST_NONFINITE;
  if (HE[HBINS - 1].cnt) flags |= ST_OVERFLOW;
  u64 U = hist_total(HN);
  const double U2 = wb_round(U);
  if (lane == 0) {
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
  if (comp < 8 && j.Bov[comp] >= 0.0) B = j.Bov[comp];
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
  int bstar = -1;
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
    for (int k = 0; k < 32; ++k) {
      const int bin = 32 * l + k;
      if (bin >= HBINS - 1) break;
      const HistBin h = HE[bin];
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
  // counts above b*
  u64 above = 0ull;
  for (int k = 0; k < 32; ++k) {
    const int bin = 32 * lane + k;
    if (bin > bstar && bin < HBINS - 1) above += HE[bin].cnt;
  }
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
  }
}

// --------------------------------------------------------------------------
// pass 2: list the energies that fall in the boundary bin b*.

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

template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass2(Job j) {
  typedef Shape<N> S;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  __shared__ double tile[S::TILE];
  const int tid = threadIdx.x, comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->resolved) return;
  const u64 prefix = st->key_prefix, mask = st->key_mask;
  u64* list = j.lists + ((size_t)comp * 2 + 0) * j.list_cap;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const double* u = j.u + (size_t)comp * j.comp_stride;
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    load_tile<T>(tile, u + e0 * n3, ne * n3, tid);
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    const long long e = e0 + el;
    double x[n];
    if (act) Fwd64<N>::stage1(tile, tile, j.tab.A, el, a, b, x);
    __syncthreads();
    if (act) Fwd64<N>::stage2(tile, j.tab.A, el, a, b);
    __syncthreads();
    double c[n];
    if (act) Fwd64<N>::stage3(tile, j.tab.A, el, a, b, c);
#pragma unroll
    for (int r = 0; r < n; ++r) {
      u64 key = 0;
      bool m = false;
      if (act) {
        const double en = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
        key = dbits(en);
        m = (key & mask) == prefix;
      }
      list_append(list, &st->list_count[0], j.list_cap, m, key, &st->flags);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// refine, level L in 2..6: histogram of the next fraction bits of the listed
// energies that match the current prefix; for L >= 3 the matching keys are
// also copied to the other list.

DEV int list_out(int L) { return ((L - 3) % 2 == 0) ? 1 : 0; }
DEV int list_in(int L) { return L == 2 ? 0 : 1 - list_out(L); }
DEV int list_members(int L) { return L == 2 ? 0 : list_out(L); }

__global__ __launch_bounds__(256) void k_refine(Job j, int L) {
  __shared__ u64 h[RBINS][2];
  const int tid = threadIdx.x, comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->resolved) return;
  const int nb = 1 << level_bits(L), sh = level_shift(L);
  const u64 fmask = (u64)(nb - 1);
  for (int k = tid; k < nb; k += 256) h[k][0] = h[k][1] = 0ull;
  __syncthreads();
  const int li = list_in(L);
  const u64* in = j.lists + ((size_t)comp * 2 + li) * j.list_cap;
  const u64 nin = st->list_count[li] < j.list_cap ? st->list_count[li] : j.list_cap;
  const u64 prefix = st->key_prefix, mask = st->key_mask;
  const int bstar = st->bstar;
  const u64 implicit = bstar ? (1ull << 52) : 0ull;
  const int lo_idx = L >= 3 ? list_out(L) : 0;
  u64* out = j.lists + ((size_t)comp * 2 + lo_idx) * j.list_cap;
  const u64 stride = (u64)gridDim.x * 256;
  // the loop trip count is the same for every lane of a wave (ballots inside)
  const u64 nin_r = (nin + 63) & ~63ull;
  for (u64 i = (u64)blockIdx.x * 256 + tid; i < nin_r; i += stride) {
    u64 key = 0;
    bool m = false;
    if (i < nin) {
      key = in[i];
      m = (key & mask) == prefix;
    }
    if (m) {
      const u64 sig = (key & M52) | implicit;
      const int sb = (int)((key >> sh) & fmask);
      atomicAdd(&h[sb][0], (1ull << 43) + (sig & M21));
      atomicAdd(&h[sb][1], sig >> 21);
    }
    if (L >= 3) list_append(out, &st->list_count[lo_idx], j.list_cap, m, key, &st->flags);
  }
  __syncthreads();
  HistBin* g = j.histL + ((size_t)(L - 2) * j.ncomp + comp) * RBINS;
  for (int k = tid; k < nb; k += 256) {
    const u64 w0 = h[k][0], w1 = h[k][1];
    if (w0 | w1) global_bin_add(g, k, w0 >> 43, w0 & M43, w1);
  }
}

// Resolve tau among <= CAP listed members of the current sub-bin by sorting
// them and scanning their significands in ascending order.
DEV void resolve_sorted(Job& j, CompState* st, int comp, int ml, int L, u64* keys, u64* slo, u64* shi,
                        int* best) {
  const int tid = threadIdx.x;
  const u64* list = j.lists + ((size_t)comp * 2 + ml) * j.list_cap;
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

__global__ __launch_bounds__(256) void k_select(Job j, int L) {
  __shared__ u64 keys[CAP];
  __shared__ u64 slo[256], shi[256];
  __shared__ int best;
  const int comp = blockIdx.x, tid = threadIdx.x;
  CompState* st = j.st + comp;
  if (st->resolved) return;
  const int ml = list_members(L);
  if (st->cur_count <= (u64)CAP) {
    resolve_sorted(j, st, comp, ml, L, keys, slo, shi, &best);
    return;
  }
  if (tid >= 64) return;
  // walk the level-L sub-bins with one wave
  const int nb = 1 << level_bits(L), sh = level_shift(L);
  const HistBin* H = j.histL + ((size_t)(L - 2) * j.ncomp + comp) * RBINS;
  const int per = nb >= 64 ? nb / 64 : 1;
  const int lane = tid;
  u128 cs = 0;
  u64 cc = 0;
  for (int k = 0; k < per; ++k) {
    const int sb = lane * per + k;
    if (sb < nb) {
      cs += bin_sum(H[sb]);
      cc += H[sb].cnt;
    }
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
  int chosen = -1;
  for (int k = 0; k < per; ++k) {
    const int sb = fl * per + k;
    if (sb >= nb) break;
    const HistBin h = H[sb];
    if (h.cnt == 0ull) continue;
    const u128 s = bin_sum(h);
    chosen = sb;
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
  for (int k = 0; k < per; ++k) {
    const int sb = lane * per + k;
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
    st->cur_count = H[chosen].cnt;
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

// --------------------------------------------------------------------------
// pass 3: compaction and verification.  Tiles are claimed in order from a
// ticket counter; each tile publishes its kept count and looks back over its
// predecessors for the exclusive prefix (single-pass decoupled look-back).

DEV u64 lb_load(const u64* p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT); }
DEV void lb_store(u64* p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }

template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_pass3(Job j) {
  typedef Shape<N> S;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS, W = S::W;
  __shared__ double su[S::TILE];
  __shared__ double sw[S::TILE];
  __shared__ LdsHist hR;
  __shared__ u64 bm[EPI * W];
  __shared__ u32 cntl[EPI];
  __shared__ u64 excl_s;
  __shared__ long long ticket_s;
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
  lh_init(hR, tid, T);
  int cur = -1;
  bool first = true;
  for (;;) {
    __syncthreads();
    if (tid == 0) ticket_s = (long long)atomicAdd(&j.ticket[0], 1u);
    __syncthreads();
    const long long tk = ticket_s;
    if (tk >= total) break;
    const int comp = (int)(tk / tiles);
    const long long t = tk % tiles;
    if (comp != cur) {
      if (cur >= 0) {
        lh_flush(hR, j.histR + (size_t)cur * HBINS, tid, T);
        __syncthreads();
        lh_init(hR, tid, T);
        __syncthreads();
      }
      cur = comp;
      first = true;
    }
    const CompState* st = j.st + comp;
    const double tau = st->tau;
    u64 voff = 0;
    for (int cc = 0; cc < comp; ++cc) voff += j.st[cc].kept;
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    const double* u = j.u + (size_t)comp * j.comp_stride;
    load_tile<T>(su, u + e0 * n3, ne * n3, tid);
    for (int k = tid; k < EPI * W; k += T) bm[k] = 0ull;
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    const long long e = e0 + el;
    double x[n];
    if (act) Fwd64<N>::stage1(su, sw, j.tab.A, el, a, b, x);
    __syncthreads();
    if (act) Fwd64<N>::stage2(sw, j.tab.A, el, a, b);
    __syncthreads();
    double c[n];
    bool keep[n];
    if (act) {
      Fwd64<N>::stage3(sw, j.tab.A, el, a, b, c);
#pragma unroll
      for (int r = 0; r < n; ++r) {
        const double en = jw(j.jac, e, j.tab.g3[(r * n + a) * n + b]) * (c[r] * c[r]);
        keep[r] = en >= tau;
        if (keep[r]) {
          const int f = (r * n + a) * n + b;
          atomicOr(&bm[el * W + (f >> 6)], 1ull << (f & 63));
        }
      }
    }
    __syncthreads();
    if (tid < EPI) {
      u32 s = 0;
      if (tid < ne)
        for (int w = 0; w < W; ++w) s += (u32)__popcll(bm[tid * W + w]);
      cntl[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
      u64 agg = 0;
      for (int k = 0; k < ne; ++k) agg += cntl[k];
      u64* lb = j.lookback + (size_t)comp * tiles;
      u64 ex = 0;
      if (t == 0) {
        lb_store(&lb[0], (2ull << 62) | agg);
      } else {
        lb_store(&lb[t], (1ull << 62) | agg);
        long long q = t - 1;
        for (;;) {
          u64 sv;
          int spins = 0;
          do {
            sv = lb_load(&lb[q]);
            if ((sv >> 62) != 0ull) break;
            __builtin_amdgcn_s_sleep(1);
          } while (++spins < SPIN_LIMIT);
          if ((sv >> 62) == 0ull) {
            atomicOr(&j.st[comp].flags, ST_SPIN);
            break;
          }
          ex += sv & M62;
          if ((sv >> 62) == 2ull) break;
          --q;
        }
        lb_store(&lb[t], (2ull << 62) | (ex + agg));
      }
      excl_s = ex;
    }
    __syncthreads();
    const u64 ex = excl_s;
    // bitmap words and offsets
    u64* gbm = j.bitmap + ((size_t)comp * E + e0) * W;
    for (int k = tid; k < ne * W; k += T) gbm[k] = bm[k];
    u64* gptr = j.elem_ptr + (size_t)comp * (E + 1);
    if (tid < ne) {
      u64 o = ex;
      for (int k = 0; k < tid; ++k) o += cntl[k];
      gptr[e0 + tid] = o;
      if (e0 + tid == E - 1) gptr[E] = o + cntl[tid];
    }
    // kept values, (element, f) order
    if (act) {
      u64 eoff = ex;
      for (int k = 0; k < el; ++k) eoff += cntl[k];
#pragma unroll
      for (int r = 0; r < n; ++r) {
        if (!keep[r]) continue;
        const int f = (r * n + a) * n + b;
        const int wi = f >> 6;
        u32 rank = 0;
        for (int w = 0; w < wi; ++w) rank += (u32)__popcll(bm[el * W + w]);
        rank += (u32)__popcll(bm[el * W + wi] & ((1ull << (f & 63)) - 1ull));
        const u64 pos = voff + eoff + rank;
        if (j.vbytes == 8)
          ((double*)j.values)[pos] = c[r];
        else
          ((float*)j.values)[pos] = (float)c[r];
      }
    }
    // inverse transform of the kept set and exact error terms
    if (act) {
      double cm[n];
#pragma unroll
      for (int r = 0; r < n; ++r) cm[r] = keep[r] ? c[r] : 0.0;
      Inv64<N>::stageA(sw, j.tab.V, el, a, b, cm);
    }
    __syncthreads();
    if (act) Inv64<N>::stageB(sw, j.tab.V, el, a, b);
    __syncthreads();
    double et[n];
    if (act) {
      double ut[n];
      Inv64<N>::stageC(sw, j.tab.V, el, a, b, ut);
      const double* w3 = j.tab.w3 + (a * n + b) * n;
      const double* pu = su + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double d = pu[i] - ut[i];
        et[i] = jw(j.jac, e, w3[i]) * (d * d);
      }
    }
    if (first) {
      if (act) {
#pragma unroll
        for (int i = 0; i < n; ++i) lh_note_max(hR, et[i]);
      }
      __syncthreads();
      if (tid == 0) lh_place(hR);
      __syncthreads();
      first = false;
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < n; ++i) lh_insert(hR, j.histR + (size_t)comp * HBINS, et[i]);
    }
  }
  __syncthreads();
  if (cur >= 0) lh_flush(hR, j.histR + (size_t)cur * HBINS, tid, T);
}

// --------------------------------------------------------------------------
// finalize (one wave per component): err2, rel, dropped energy.

__global__ __launch_bounds__(64) void k_finalize(Job j) {
  const int comp = blockIdx.x, lane = threadIdx.x;
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

// --------------------------------------------------------------------------
// decompress: bitmap + offsets + values -> nodal field (FP64 fixed order).

template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_decompress(Job j, void* out, int out_fp64) {
  typedef Shape<N> S;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS, W = S::W;
  __shared__ double sw[S::TILE];
  __shared__ u64 bm[EPI * W];
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
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
    if (act) {
      const u64 base = voff + j.elem_ptr[(size_t)comp * (E + 1) + e0 + el];
      double cm[n];
#pragma unroll
      for (int r = 0; r < n; ++r) {
        const int f = (r * n + a) * n + b;
        const int wi = f >> 6;
        const u64 word = bm[el * W + wi];
        cm[r] = 0.0;
        if ((word >> (f & 63)) & 1ull) {
          u32 rank = 0;
          for (int w = 0; w < wi; ++w) rank += (u32)__popcll(bm[el * W + w]);
          rank += (u32)__popcll(word & ((1ull << (f & 63)) - 1ull));
          cm[r] = j.vbytes == 8 ? ((const double*)j.values)[base + rank]
                                : (double)((const float*)j.values)[base + rank];
        }
      }
      Inv64<N>::stageA(sw, j.tab.V, el, a, b, cm);
    }
    __syncthreads();
    if (act) Inv64<N>::stageB(sw, j.tab.V, el, a, b);
    __syncthreads();
    double ut[n];
    if (act) Inv64<N>::stageC(sw, j.tab.V, el, a, b, ut);
    __syncthreads();
    if (act) {
      double* pout = sw + el * n3 + (a * n + b) * n;
#pragma unroll
      for (int i = 0; i < n; ++i) pout[i] = ut[i];
    }
    __syncthreads();
    const size_t obase = ((size_t)comp * E + e0) * n3;
    if (out_fp64) {
      double* o = (double*)out + obase;
      for (int k = tid; k < ne * n3; k += T) o[k] = sw[k];
    } else {
      float* o = (float*)out + obase;
      for (int k = tid; k < ne * n3; k += T) o[k] = (float)sw[k];
    }
  }
}

// forward transform only (FP64 fixed order), coefficients to global memory
template <int N>
__global__ __launch_bounds__(Shape<N>::THREADS) void k_forward(Job j, double* coef) {
  typedef Shape<N> S;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, EPI = S::EPI, T = S::THREADS;
  __shared__ double tile[S::TILE];
  const int tid = threadIdx.x;
  const int el = tid / n2, a = (tid % n2) / n, b = tid % n;
  const long long E = j.n_elem;
  const long long tiles = (E + EPI - 1) / EPI;
  const long long total = tiles * j.ncomp;
  for (long long tk = blockIdx.x; tk < total; tk += gridDim.x) {
    const int comp = (int)(tk / tiles);
    const long long t = tk % tiles;
    const long long e0 = t * EPI;
    const int ne = (int)((E - e0) < EPI ? (E - e0) : EPI);
    __syncthreads();
    load_tile<T>(tile, j.u + (size_t)comp * j.comp_stride + e0 * n3, ne * n3, tid);
    __syncthreads();
    const bool act = tid < S::ACT && el < ne;
    double x[n];
    if (act) Fwd64<N>::stage1(tile, tile, j.tab.A, el, a, b, x);
    __syncthreads();
    if (act) Fwd64<N>::stage2(tile, j.tab.A, el, a, b);
    __syncthreads();
    double c[n];
    if (act) Fwd64<N>::stage3(tile, j.tab.A, el, a, b, c);
    __syncthreads();
    if (act) {
      double* col = tile + el * n3 + a * n + b;
#pragma unroll
      for (int r = 0; r < n; ++r) col[r * n2] = c[r];
    }
    __syncthreads();
    double* o = coef + ((size_t)comp * E + e0) * n3;
    for (int k = tid; k < ne * n3; k += T) o[k] = tile[k];
  }
}

// --------------------------------------------------------------------------
// host launchers with a switch over the compile-time order

int words_per_elem(int order) {
  const int n = order + 1, n3 = n * n * n;
  return (n3 + 63) / 64;
}

#define ISR_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

static int epi_of(int order) {
  switch (order) {
#define CASE(NN) \
  case NN:       \
    return Shape<NN>::EPI;
    ISR_ORDERS(CASE)
#undef CASE
  }
  return 1;
}

int tiles_per_comp(int order, long long n_elem) {
  const int epi = epi_of(order);
  return (int)((n_elem + epi - 1) / epi);
}

hipError_t launch_pass1(const Job& j, int gx, hipStream_t s) {
  switch (j.order) {
#define CASE(NN)                                                                                       \
  case NN:                                                                                             \
    hipLaunchKernelGGL(k_pass1<NN>, dim3(gx, j.ncomp), dim3(Shape<NN>::THREADS), 0, s, j);            \
    break;
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_select1(const Job& j, hipStream_t s) {
  hipLaunchKernelGGL(k_select1, dim3(j.ncomp), dim3(64), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_pass2(const Job& j, int gx, hipStream_t s) {
  switch (j.order) {
#define CASE(NN)                                                                                       \
  case NN:                                                                                             \
    hipLaunchKernelGGL(k_pass2<NN>, dim3(gx, j.ncomp), dim3(Shape<NN>::THREADS), 0, s, j);            \
    break;
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_refine(const Job& j, int L, int gx, hipStream_t s) {
  hipLaunchKernelGGL(k_refine, dim3(gx, j.ncomp), dim3(256), 0, s, j, L);
  return hipGetLastError();
}

hipError_t launch_select(const Job& j, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(j.ncomp), dim3(256), 0, s, j, L);
  return hipGetLastError();
}

hipError_t launch_pass3(const Job& j, int grid, hipStream_t s) {
  switch (j.order) {
#define CASE(NN)                                                                                       \
  case NN:                                                                                             \
    hipLaunchKernelGGL(k_pass3<NN>, dim3(grid), dim3(Shape<NN>::THREADS), 0, s, j);                   \
    break;
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const Job& j, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(j.ncomp), dim3(64), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_decompress(const Job& j, void* out, int out_fp64, int grid, hipStream_t s) {
  switch (j.order) {
#define CASE(NN)                                                                                       \
  case NN:                                                                                             \
    hipLaunchKernelGGL(k_decompress<NN>, dim3(grid), dim3(Shape<NN>::THREADS), 0, s, j, out, out_fp64); \
    break;
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const Job& j, void* coef, int grid, hipStream_t s) {
  switch (j.order) {
#define CASE(NN)                                                                                       \
  case NN:                                                                                             \
    hipLaunchKernelGGL(k_forward<NN>, dim3(grid), dim3(Shape<NN>::THREADS), 0, s, j, (double*)coef);  \
    break;
    ISR_ORDERS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace isr
