// Per-element cut: a variant of the lossy step's selection in which every
// element is cut alone by the plain value rule, at its own share of the
// budget (Sec. IV-B: the lossy step's sorting kernels; the global cut's
// threshold rule applied inside one element).  FP64 path.
//
// One wavefront per element.  Its norm terms and energies are formed from
// the field and the FP64 coefficients (isr_forward's), and the element's
// threshold is found by a binary search over the bit patterns of the
// energies (monotone for non-negative doubles), which stops once no energy
// lies strictly inside the interval.  Each probe decides RN(exact sum of
// energies below the key) <= B_e: an FP64 wave sum with a rigorous error
// bound settles almost every probe, and the rest are summed exactly.  Exact
// sums: every lane splits its terms by error-free extraction against 2^m >=
// the wave's largest term into three FP64 sums (exact), their wave totals
// form one 192-bit integer in a wave big integer (X units of 2^-1075), and
// the rare remainders (bits far below 2^m) go through 32-bit digits in LDS;
// the result is rounded once.  The workgroup adds every element's exact norm
// and dropped energy into per-component digit totals, and the finishing
// kernel rounds the component totals.  Compaction, the inverse and the exact
// error check are pass 3 of the general pipeline, reading the per-element
// thresholds.
#include "isr.h"
#include "isr_common.cuh"
#include "isr_xsum.cuh"

namespace isr {

namespace {

constexpr int ED = 68;       // digits of one element's sum (top term bit < 2^2099, 12 bits of count)
constexpr int GD = 128;      // digits of a component total (the 64 words of a wave big integer)
constexpr int EC_WAVES = 4;  // wavefronts per workgroup
constexpr u64 INF_KEY = 0x7ff0000000000000ull;

DEV double jw1(const double* jac, long long e, double t) { return jac ? jac[e] * t : t; }

struct ElemLds {
  u64 d[EC_WAVES][ED];             // per wavefront: the sum being formed
  u64 tot[ISR_MAX_COMP][2][GD];    // per component: norm (0) and dropped energy (1)
  u64 kept[ISR_MAX_COMP];
};

// LDS operations of one wavefront complete in issue order; the fence keeps
// the compiler from moving the accesses around each other.
DEV void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

DEV void ed_clear(u64* D) {
  const int l = lane_id();
  D[l] = 0ull;
  if (l < ED - 64) D[64 + l] = 0ull;
  wave_order();
}

// Adds a finite x >= 0: its significand at X-unit shift max(E, 1) spans
// three 32-bit digits.
DEV void ed_add(u64* D, double x) {
  const u64 bits = dbits(x);
  if (bits == 0ull) return;
  const int E = (int)(bits >> 52);
  const u64 sig = (bits & M52) | (E ? (1ull << 52) : 0ull);
  const int sh = E ? E : 1;
  const int d = sh >> 5, r = sh & 31;
  const u64 lo = sig << r;
  const u64 hi = r ? (sig >> (64 - r)) : 0ull;
  atomicAdd((unsigned long long*)&D[d], (unsigned long long)(lo & 0xffffffffull));
  atomicAdd((unsigned long long*)&D[d + 1], (unsigned long long)(lo >> 32));
  if (hi) atomicAdd((unsigned long long*)&D[d + 2], (unsigned long long)hi);
}

// Digits (each below 2^64, digit i of weight 2^(32 i)) as a wave big
// integer: lane l holds bits [64 l, 64 l + 64).
DEV u64 digits_to_words(u64 a, u64 b) {
  const u64 lo = a + (b << 32);
  const u64 hi = (b >> 32) + (lo < a ? 1ull : 0ull);
  u64 w = lo;
  u64 up = shfl_up64(hi, 1);
  if (lane_id() == 0) up = 0ull;
  wb_add(w, up);
  return w;
}

DEV u64 ed_words(const u64* D) {
  wave_order();
  const int l = lane_id();
  const u64 a = 2 * l < ED ? D[2 * l] : 0ull;
  const u64 b = 2 * l + 1 < ED ? D[2 * l + 1] : 0ull;
  return digits_to_words(a, b);
}

// A wave big integer (each word split in two 32-bit digits) into totals.
DEV void tot_add(u64* T, u64 w) {
  if (w == 0ull) return;
  const int l = lane_id();
  atomicAdd((unsigned long long*)&T[2 * l], (unsigned long long)(w & 0xffffffffull));
  atomicAdd((unsigned long long*)&T[2 * l + 1], (unsigned long long)(w >> 32));
}

DEV u64 wmax64(u64 v);

// X-unit wave big integer of the exact sum of the terms x[k] with take[k]
// (finite, >= 0) over the wave's lanes.
template <int CNT>
DEV u64 exact_words(const double (&x)[CNT], const bool (&take)[CNT], u64* D) {
  u64 mk = 0ull;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const u64 b = take[k] ? dbits(x[k]) : 0ull;
    mk = b > mk ? b : mk;
  }
  mk = wmax64(mk);
  if (mk == 0ull) return 0ull;
  // every term is below 2^m (exponent of the largest term plus one)
  int m = (int)(mk >> 52) - 1022;
  m = m < XM_MIN ? XM_MIN : (m > XM_MAX ? XM_MAX : m);
  constexpr int h = 7;  // a lane adds at most 64 = 2^(h-1) terms
  const XParm P = xparm(m, h);
  XAcc A = {0.0, 0.0, 0.0};
  bool rem = false;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    double left;
    rem = xadd_left(A, P, take[k] ? x[k] : 0.0, left) || rem;
  }
  long long K[3];
  xints(A, P, K);
  I192 z = {{0ull, 0ull, 0ull}};
  const int sft[3] = {107 - 2 * h, 53 - h, 0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    __int128 t = (__int128)K[i];
    for (int mm = 32; mm > 0; mm >>= 1) t += shfl_xor128(t, mm);
    i192_add_shl(z, t, sft[i]);
  }
  // z counts units u3 = 2^(m + 3h - 159), i.e. X units shifted by sh (>= 61)
  const int sh = m + 3 * h - 159 + 1075;
  u64 w = part_at(z.w[0], z.w[1], sh);
  wb_add(w, part_at(z.w[2], 0ull, sh + 128));
  if (ballot(rem)) {
    ed_clear(D);
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      XAcc scratch = {0.0, 0.0, 0.0};
      double left = 0.0;
      if (xadd_left(scratch, P, take[k] ? x[k] : 0.0, left) && left != 0.0) ed_add(D, left);
    }
    wb_add(w, ed_words(D));
  }
  return w;
}

DEV double wsum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

DEV u64 wmin64(u64 v) {
  for (int m = 32; m > 0; m >>= 1) {
    const u64 o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

DEV u64 wmax64(u64 v) {
  for (int m = 32; m > 0; m >>= 1) {
    const u64 o = shfl_xor64(v, m);
    v = o > v ? o : v;
  }
  return v;
}

// RN(exact sum of the energies whose key is below K) <= B, the same answer
// in every lane.  Padding slots carry key ~0 and never count.  The FP64 sum
// of C non-negative terms, in any order, is within (C - 1) 2^-53 of the
// exact sum (first order); twice that settles the probe when B (or the
// successor of B) lies outside the band.
template <int CNT>
DEV bool ec_feasible(const double (&x)[CNT], const u64 (&key)[CNT], u64 K, double B, double succB, u64* D) {
  double s = 0.0;
  int c = 0;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const bool in = key[k] < K;
    s = s + (in ? x[k] : 0.0);
    c += __popcll(ballot(in));
  }
  const double S = wsum(s);
  const double C = (double)c;
  const double bound = ((2.0 * C) * 0x1p-53) * S;
  if (S + bound <= B) return true;
  if (S - bound > succB) return false;
  bool in[CNT];
#pragma unroll
  for (int k = 0; k < CNT; ++k) in[k] = key[k] < K;
  return wb_round(exact_words<CNT>(x, in, D)) <= B;
}

}  // namespace

struct ElemScale {
  double s[ISR_MAX_COMP];  // budget scale per component (1 until a repair)
};

template <int N>
__global__ __launch_bounds__(256) void k_elemsel(Job j, const double* coef, double* tau_out, u64* G, ElemScale sc) {
  constexpr int n = N + 1, n3 = n * n * n, CNT = (n3 + 63) / 64;
  __shared__ ElemLds L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < ISR_MAX_COMP * 2 * GD; i += 256) (&L.tot[0][0][0])[i] = 0ull;
  if (tid < ISR_MAX_COMP) L.kept[tid] = 0ull;
  __syncthreads();
  u64* D = L.d[wv];
  const long long E = j.n_elem, pairs = E * j.ncomp;
  const double tt = j.tol * j.tol;
  for (long long p = (long long)blockIdx.x * EC_WAVES + wv; p < pairs; p += (long long)gridDim.x * EC_WAVES) {
    const int comp = (int)(p / E);
    const long long e = p - (long long)comp * E;
    const double* ue = j.u + (size_t)comp * j.comp_stride + (size_t)e * n3;
    const double* ce = coef + (size_t)p * n3;
    double t[CNT], x[CNT];
    u64 key[CNT];
    bool badu = false, bad = false;
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const int f = lane + 64 * k;
      if (f < n3) {
        const double uv = ue[f], cv = ce[f];
        t[k] = jw1(j.jac, e, j.tab.w3[f]) * (uv * uv);
        x[k] = jw1(j.jac, e, j.tab.g3[f]) * (cv * cv);
        key[k] = dbits(x[k]);
        badu = badu || !__builtin_isfinite(uv);
        bad = bad || !(t[k] >= 0.0 && t[k] <= 0x1.fffffffffffffp+1023) ||
              !(x[k] >= 0.0 && x[k] <= 0x1.fffffffffffffp+1023);
      } else {
        t[k] = 0.0;
        x[k] = 0.0;
        key[k] = ~0ull;
      }
    }
    const u64 ub = ballot(badu), xb = ballot(bad);
    if (ub | xb) {  // non-finite field value, or an energy or norm term out of range
      if (lane == 0) {
        atomicOr(&j.st[comp].flags, ub ? (int)ST_NONFINITE : (int)ST_OVERFLOW);
        tau_out[p] = __builtin_inf();
      }
      continue;
    }
    // the element's norm, exactly, and its budget
    bool valid[CNT];
#pragma unroll
    for (int k = 0; k < CNT; ++k) valid[k] = lane + 64 * k < n3;
    u64 w = exact_words<CNT>(t, valid, D);
    const double U2e = wb_round(w);
    tot_add(L.tot[comp][0], w);
    const double B = (tt * U2e) * sc.s[comp];
    const double succB = __longlong_as_double((long long)(dbits(B) + 1ull));
    // the element's threshold
    u64 kt;
    if (ec_feasible<CNT>(x, key, INF_KEY, B, succB, D)) {
      kt = INF_KEY;  // everything fits the budget: +inf, nothing kept
    } else {
      u64 mn = ~0ull, mx = 0ull;
#pragma unroll
      for (int k = 0; k < CNT; ++k) {
        if (lane + 64 * k < n3) {
          mn = key[k] < mn ? key[k] : mn;
          mx = key[k] > mx ? key[k] : mx;
        }
      }
      u64 lo = wmin64(mn), hi = wmax64(mx) + 1ull;  // S(lo) = 0 <= B; S(hi) = the total > B
      while (hi - lo > 1ull) {
        // no energy strictly between lo and hi: then S(hi) = S(lo) plus the
        // energies at key lo, and S(lo) <= B < S(hi) makes lo an energy's key
        // (the answer); bisection stops here long before the keys run out
        bool inside = false;
#pragma unroll
        for (int k = 0; k < CNT; ++k) inside = inside || (key[k] > lo && key[k] < hi);
        if (!ballot(inside)) break;
        const u64 mid = lo + ((hi - lo) >> 1);
        if (ec_feasible<CNT>(x, key, mid, B, succB, D))
          lo = mid;
        else
          hi = mid;
      }
      kt = lo;  // S(lo) <= B < S(lo + 1): lo is the key of an energy
    }
    // dropped energy, exactly, and the kept count
    bool drop[CNT];
    u64 kc = 0;
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      drop[k] = valid[k] && key[k] < kt;
      kc += (valid[k] && !drop[k]) ? 1ull : 0ull;
    }
    w = exact_words<CNT>(x, drop, D);
    tot_add(L.tot[comp][1], w);
    kc = wave_sum64(kc);
    if (lane == 0) {
      atomicAdd((unsigned long long*)&L.kept[comp], (unsigned long long)kc);
      tau_out[p] = __longlong_as_double((long long)kt);
    }
  }
  __syncthreads();
  for (int i = tid; i < j.ncomp * 2 * GD; i += 256) {
    const u64 v = (&L.tot[0][0][0])[i];
    if (v) atomicAdd((unsigned long long*)&G[i], (unsigned long long)v);
  }
  if (tid < j.ncomp && L.kept[tid]) atomicAdd((unsigned long long*)&j.st[tid].kept, (unsigned long long)L.kept[tid]);
}

// Component totals: U2 and the dropped energy rounded from their digits;
// the threshold is per element (NaN here), and the selection is final.
__global__ __launch_bounds__(64) void k_elemfin(Job j, const u64* G) {
  const int comp = blockIdx.x, l = lane_id();
  double v[2];
  for (int k = 0; k < 2; ++k) {
    const u64* T = G + ((size_t)comp * 2 + k) * GD;
    v[k] = wb_round(digits_to_words(T[2 * l], T[2 * l + 1]));
  }
  if (l == 0) {
    CompState* st = j.st + comp;
    st->U2 = v[0];
    st->B = (j.tol * j.tol) * v[0];
    st->tau = __builtin_nan("");
    st->dropped = v[1];
    st->resolved = 1;
    st->bstar = -1;
  }
}

size_t elemcut_digit_bytes(int ncomp) { return (size_t)ncomp * 2 * GD * sizeof(u64); }

hipError_t launch_elemcut(const Job& j, const double* coef, double* tau, u64* G, const double* scale, int grid,
                          hipStream_t s) {
  ElemScale sc;
  for (int k = 0; k < ISR_MAX_COMP; ++k) sc.s[k] = k < j.ncomp ? scale[k] : 1.0;
  switch (j.order) {
#define EC_CASE(NN)                                                                              \
  case NN:                                                                                       \
    hipLaunchKernelGGL((k_elemsel<NN>), dim3(grid), dim3(256), 0, s, j, coef, tau, G, sc);      \
    break;
    EC_CASE(1) EC_CASE(2) EC_CASE(3) EC_CASE(4) EC_CASE(5) EC_CASE(6) EC_CASE(7) EC_CASE(8)
    EC_CASE(9) EC_CASE(10) EC_CASE(11) EC_CASE(12) EC_CASE(13) EC_CASE(14) EC_CASE(15)
#undef EC_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_elemfin, dim3(j.ncomp), dim3(64), 0, s, j, (const u64*)G);
  return hipGetLastError();
}

}  // namespace isr
