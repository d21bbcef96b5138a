// Exact sums without atomics on the hot path, shared by the streaming
// passes (isr_engine.cuh) and the order-independent kernels (isr_select.hip).
//
// Every lane splits each non-negative term x <= M = 2^m into three parts on
// fixed grids by error-free extraction against fixed powers of two (Rump,
// Ogita and Oishi, "Accurate floating-point summation part I", SIAM J. Sci.
// Comput. 31(1), 2008, Alg. 3.2) and keeps three FP64 running sums, which
// stay exact while a lane adds at most 2^(h-1) terms.  A term that leaves a
// remainder (far below M, or above M) goes to the global exponent bins.
// Workgroups publish the three sums as integers; the consumer adds them up
// as 128-bit integers and writes the exact total into exponent bins.  On the
// FP64 path every term is split this way; on the MFMA paths a lane first adds
// its terms in a fixed FP64 order and only that total is split (xadd_sum).
#pragma once

#include "isr_common.cuh"

namespace isr {

typedef double d2 __attribute__((ext_vector_type(2)));

// ---- exact sums by error-free extraction -------------------------------------
constexpr int XM_MIN = -876;  // keeps every extraction unit a normal number
constexpr int XM_MAX = 800;   // keeps the three 64-bit words of a total below bin 2047
constexpr int XH_MIN = 7, XH_MAX = 20;

// Units (exponents of 2) of the three parts: u1 = m + h - 52, u2 = m + 2h - 106,
// u3 = m + 3h - 159.  A lane may add at most 2^(h-1) terms.
struct XParm {
  double S1, S2, S3, u3, M;
  int m, h;
};

// 2^k for a normal exponent k, built from its bits (scalar instructions, so the
// parameters stay in scalar registers)
DEV double pow2(int k) { return __longlong_as_double((long long)(k + 1023) << 52); }

DEV XParm xparm(int m, int h) {
  XParm P;
  P.m = m;
  P.h = h;
  P.M = pow2(m);
  P.S1 = pow2(m + h);
  P.S2 = pow2(m + 2 * h - 53);
  P.S3 = pow2(m + 3 * h - 106);
  P.u3 = pow2(m + 3 * h - 159);
  return P;
}

struct XAcc {
  double a1, a2, a3;
};

// One term straight into the exact global exponent bins.
DEV void slow_bin(HistBin* g, double v) {
  const u64 bits = dbits(v);
  if (bits == 0ull) return;
  const int E = bits_exp(bits);
  u64 sig = (bits & M52) | (E ? (1ull << 52) : 0ull);
  if (E == 2047) sig = 0ull;
  global_bin_add(g, E, 1ull, sig & M21, sig >> 21);
}

// Branch-free form: adds x to the three sums and returns what is left for
// the exact global bins (0 for almost every term; x itself when x is not in
// [0, M], which includes Inf and NaN).
// 0 <= x < M = 2^m by the high words alone (M's low word is zero): a set
// sign bit, Inf and NaN fail, and so does x == M, which then takes the exact
// slow path like any term out of range.
DEV bool xin(const XParm& P, double x) {
  return (u32)((u64)__double_as_longlong(x) >> 32) < (u32)((u64)__double_as_longlong(P.M) >> 32);
}

DEV double xadd_r(XAcc& A, const XParm& P, double x) {
  const bool in = xin(P, x);
  const double y = in ? x : 0.0;
  const double q1 = (P.S1 + y) - P.S1;
  const double r1 = y - q1;
  const double q2 = (P.S2 + r1) - P.S2;
  const double r2 = r1 - q2;
  const double t3 = (P.S3 + r2) - P.S3;
  const double q3 = t3 > r2 ? t3 - P.u3 : t3;
  A.a1 = A.a1 + q1;
  A.a2 = A.a2 + q2;
  A.a3 = A.a3 + q3;
  return in ? r2 - q3 : x;
}

// xadd_r with its result split for the caller's test: true when something is
// left for the exact global bins, and then `left` is what (the selection
// that forms it is only needed on that rarely taken branch).
DEV bool xadd_left(XAcc& A, const XParm& P, double x, double& left) {
  const bool in = xin(P, x);
  const double y = in ? x : 0.0;
  const double q1 = (P.S1 + y) - P.S1;
  const double r1 = y - q1;
  const double q2 = (P.S2 + r1) - P.S2;
  const double r2 = r1 - q2;
  const double t3 = (P.S3 + r2) - P.S3;
  const double q3 = t3 > r2 ? t3 - P.u3 : t3;
  A.a1 = A.a1 + q1;
  A.a2 = A.a2 + q2;
  A.a3 = A.a3 + q3;
  const double r3 = r2 - q3;
  left = in ? r3 : x;
  return !in || r3 != 0.0;
}

// A lane's fixed-order FP64 sum s of at most 2^(h-1) terms in [0, M] (so
// s <= 2^(m+h-1)) added to the three sums, exactly down to u3; returns what
// is left for the global bins: the part below u3 (0 <= r < 2 u3), or s itself
// when it is out of that range (Inf and NaN included).
DEV double xadd_sum(XAcc& A, const XParm& P, double s) {
  const bool in = s >= 0.0 && s <= 0.5 * P.S1;
  const double y = in ? s : 0.0;
  const double q1 = (P.S1 + y) - P.S1;
  const double r1 = y - q1;
  const double q2 = (P.S2 + r1) - P.S2;
  const double r2 = r1 - q2;
  const double t3 = (P.S3 + r2) - P.S3;
  const double q3 = t3 > r2 ? t3 - P.u3 : t3;
  A.a1 = A.a1 + q1;
  A.a2 = A.a2 + q2;
  A.a3 = A.a3 + q3;
  return in ? r2 - q3 : s;
}

// x = q1 + q2 + q3 + r3: q_k on the grid of u_k (|q1| <= M, |q2| <= u1,
// |q3| <= u2), the last part rounded down so that 0 <= r3 < 2 u3.
DEV void xadd(XAcc& A, const XParm& P, double x, HistBin* g) {
  if (!(x >= 0.0 && x <= P.M)) {
    slow_bin(g, x);
    return;
  }
  const double q1 = (P.S1 + x) - P.S1;
  const double r1 = x - q1;
  const double q2 = (P.S2 + r1) - P.S2;
  const double r2 = r1 - q2;
  double q3 = (P.S3 + r2) - P.S3;
  if (q3 > r2) q3 = q3 - P.u3;
  const double r3 = r2 - q3;
  A.a1 = A.a1 + q1;
  A.a2 = A.a2 + q2;
  A.a3 = A.a3 + q3;
  if (r3 != 0.0) slow_bin(g, r3);
}

// The three sums as integers in their units (exact: |sum| < 2^53 units).
DEV void xints(const XAcc& A, const XParm& P, long long (&k)[3]) {
  k[0] = (long long)ldexp(A.a1, -(P.m + P.h - 52));
  k[1] = (long long)ldexp(A.a2, -(P.m + 2 * P.h - 106));
  k[2] = (long long)ldexp(A.a3, -(P.m + 3 * P.h - 159));
}

// 192-bit two's complement integer.
struct I192 {
  u64 w[3];
};

DEV void i192_add_shl(I192& z, __int128 v, int sh) {  // z += v << sh, 0 <= sh < 128
  const unsigned __int128 uv = (unsigned __int128)v;
  u64 a[3] = {(u64)uv, (u64)(uv >> 64), v < 0 ? ~0ull : 0ull};
  while (sh >= 64) {
    a[2] = a[1];
    a[1] = a[0];
    a[0] = 0ull;
    sh -= 64;
  }
  if (sh) {
    a[2] = (a[2] << sh) | (a[1] >> (64 - sh));
    a[1] = (a[1] << sh) | (a[0] >> (64 - sh));
    a[0] = a[0] << sh;
  }
  u64 c = 0;
  for (int k = 0; k < 3; ++k) {
    const u64 s = z.w[k] + a[k];
    const u64 c1 = s < z.w[k];
    const u64 s2 = s + c;
    const u64 c2 = s2 < s;
    z.w[k] = s2;
    c = c1 | c2;
  }
}

// Adds v (< 2^85) units of bin b to the global bins.  The bin also counts
// one term: readers skip bins whose count is zero (the counts of these bins,
// all below the boundary bin, are never used otherwise).
DEV void add_piece(HistBin* g, int b, unsigned __int128 v) {
  if (v == 0) return;
  const u64 lo = (u64)v & M21;
  const u64 hi = (u64)(v >> 21);
  atomicAdd(&g[b].cnt, 1ull);
  if (lo) atomicAdd(&g[b].lo, lo);
  if (hi) atomicAdd(&g[b].hi, hi);
}

// Exact total of three integer sums (units u1, u2, u3 of XParm(m, h)) as bins.
// btop < 0: three 64-bit words at the bins of u3, u3 * 2^64, u3 * 2^128;
// btop >= 0: all of it in bins <= btop (the part above bit btop - b3 in btop).
DEV void emit_total(HistBin* g, const __int128 (&K)[3], int m, int h, int btop) {
  I192 z = {{0ull, 0ull, 0ull}};
  i192_add_shl(z, K[0], 107 - 2 * h);
  i192_add_shl(z, K[1], 53 - h);
  i192_add_shl(z, K[2], 0);
  const int b3 = m + 3 * h + 916;  // bin whose unit is u3
  if (btop < 0) {
    for (int k = 0; k < 3; ++k) add_piece(g, b3 + 64 * k, z.w[k]);
    return;
  }
  const int d = btop - b3;  // 46..85 for the window placements used
  const unsigned __int128 lo128 = ((unsigned __int128)z.w[1] << 64) | z.w[0];
  const unsigned __int128 mask = d >= 128 ? ~(unsigned __int128)0 : (((unsigned __int128)1 << d) - 1);
  add_piece(g, b3, lo128 & mask);
  // z >> d (fits 85 bits: the total is below 2^32 terms of at most M each)
  unsigned __int128 hi128;
  if (d < 64)
    hi128 = (lo128 >> d) | ((unsigned __int128)z.w[2] << (128 - d));
  else
    hi128 = (((unsigned __int128)z.w[2] << 64) | z.w[1]) >> (d - 64);
  add_piece(g, btop, hi128);
}

DEV long long wave_sum_i64(long long v) { return (long long)wave_sum64((u64)v); }

DEV double wave_sum_f64(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Workgroup of 256: sums `cnt` signed 64-bit values per thread into out[k]
// (thread 0 holds the totals afterwards in red[0][k]).
template <int CNT>
DEV void block_sum_i64(long long (&v)[CNT], long long (*red)[8], int tid) {
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const long long s = wave_sum_i64(v[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < CNT; ++k) red[0][k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
  }
  __syncthreads();
}

DEV __int128 shfl_xor128(__int128 v, int m) {
  const unsigned __int128 u = (unsigned __int128)v;
  const u64 lo = shfl_xor64((u64)u, m), hi = shfl_xor64((u64)(u >> 64), m);
  return (__int128)(((unsigned __int128)hi << 64) | lo);
}

// Workgroup of 256: totals of fields 0..F-1 over `count` rows of `stride`
// 64-bit signed values starting at base (row r, field f at base[r * stride +
// f]), as 128-bit integers, in every thread.  Every field of a row is loaded
// at once, so the workgroup waits for memory once.  red: [4][F] of LDS.
template <int F>
DEV void block_totals(const long long* base, int count, int stride, __int128 (&tot)[F], __int128 (*red)[F], int tid) {
  const int lane = tid & 63, wv = tid >> 6;
  __int128 p[F];
#pragma unroll
  for (int f = 0; f < F; ++f) p[f] = 0;
  for (int r = tid; r < count; r += 256) {
    long long v[F];
#pragma unroll
    for (int f = 0; f < F; ++f) v[f] = base[(size_t)r * stride + f];
#pragma unroll
    for (int f = 0; f < F; ++f) p[f] += (__int128)v[f];
  }
#pragma unroll
  for (int f = 0; f < F; ++f)
    for (int m = 32; m > 0; m >>= 1) p[f] += shfl_xor128(p[f], m);
  if (lane == 0)
#pragma unroll
    for (int f = 0; f < F; ++f) red[wv][f] = p[f];
  __syncthreads();
#pragma unroll
  for (int f = 0; f < F; ++f) tot[f] = red[0][f] + red[1][f] + red[2][f] + red[3][f];
  __syncthreads();
}

// Last workgroup of a component to finish (returns true in every thread of
// that workgroup, after an acquire fence).
DEV bool last_block(u32* counter, int* flag_lds, int nblocks) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *flag_lds = atomicAdd(counter, 1u) == (u32)(nblocks - 1);
  __syncthreads();
  const bool last = *flag_lds != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace isr
