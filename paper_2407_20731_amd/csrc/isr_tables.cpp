// GLL / Legendre tables for order N, computed on the host in binary128
// (__float128, 113-bit significand) and rounded once to FP64 (round to
// nearest even).  Textbook spectral-element quantities:
//   xi      GLL nodes: -1, the roots of P_N', +1 (Newton on P_N', using the
//           Legendre ODE for P_N'')
//   w_i     = 2 / (N (N+1) P_N(xi_i)^2)
//   V[i][k] = P_k(xi_i)                   (standard Legendre, P_k(1) = 1)
//   gamma_k = 2/(2k+1) for k < N, 2/N for k = N   (discrete GLL norms)
//   A[p][i] = P_p(xi_i) w_i / gamma_p     (= V^-1 by discrete orthogonality)
//   w3[k][j][i] = w_k w_j w_i,  g3[r][q][p] = gamma_r gamma_q gamma_p
// gamma and g3 are exact rationals 2/d and 8/D with integer d, D < 2^53, so
// one IEEE division gives their correctly rounded values directly.
#include <cmath>
#include <cstring>

#include "isr_internal.h"

namespace isr {

typedef __float128 q128;

static void legendre_all(int kmax, q128 x, q128* P) {
  P[0] = 1;
  if (kmax >= 1) P[1] = x;
  for (int k = 1; k < kmax; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

static q128 qabs(q128 x) { return x < 0 ? -x : x; }

// Round to FP64; an exact zero is +0 (the recurrence can produce -0 at xi = 0).
static double rnd(q128 x) {
  double d = (double)x;
  return d == 0.0 ? 0.0 : d;
}

bool host_tables(int N, HostTables* t) {
  if (N < 1 || N > 15 || !t) return false;
  const int n = N + 1;
  std::memset(t, 0, sizeof(*t));
  t->N = N;
  q128 xs[16], ws[16], P[17];
  xs[0] = -1;
  xs[N] = 1;
  for (int i = 1; i < N; ++i) {
    q128 x = -std::cos(M_PI * i / N);  // Chebyshev-Gauss-Lobatto start
    for (int it = 0; it < 100; ++it) {
      legendre_all(N, x, P);
      q128 one_m = 1 - x * x;
      q128 dP = N * (P[N - 1] - x * P[N]) / one_m;
      q128 d2P = (2 * x * dP - N * (N + 1) * P[N]) / one_m;
      q128 step = dP / d2P;
      x -= step;
      if (qabs(step) < (q128)1e-33) break;
    }
    xs[i] = x;
  }
  for (int i = 0; i < n / 2; ++i) {  // exact symmetry
    q128 a = (xs[N - i] - xs[i]) / 2;
    xs[i] = -a;
    xs[N - i] = a;
  }
  if (N % 2 == 0) xs[N / 2] = 0;
  q128 Pk[16][17];
  for (int i = 0; i < n; ++i) {
    legendre_all(N, xs[i], Pk[i]);
    ws[i] = (q128)2 / ((q128)(N * (N + 1)) * Pk[i][N] * Pk[i][N]);
  }
  long long gden[16];  // gamma_k = 2 / gden[k]
  for (int k = 0; k < n; ++k) gden[k] = (k < N) ? (2 * k + 1) : N;
  for (int i = 0; i < n; ++i) {
    t->xi[i] = rnd(xs[i]);
    t->w[i] = rnd(ws[i]);
    t->gamma[i] = 2.0 / (double)gden[i];
    for (int k = 0; k < n; ++k) {
      t->V[i * n + k] = rnd(Pk[i][k]);
      // A[p][i] with p = k: P_p(xi_i) w_i / gamma_p = P_p(xi_i) w_i gden[p] / 2
      t->A[k * n + i] = rnd(Pk[i][k] * ws[i] * (q128)gden[k] / 2);
    }
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) {
        int idx = (a * n + b) * n + c;
        t->w3[idx] = rnd(ws[a] * ws[b] * ws[c]);
        t->g3[idx] = 8.0 / (double)(gden[a] * gden[b] * gden[c]);
      }
  return true;
}

}  // namespace isr
