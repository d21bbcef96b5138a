/*
 * isr_cpu.c -- a fast FP64 CPU implementation of the in-situ lossy step, the
 * multi-core baseline that the GPU library is compared with (arXiv
 * 2407.20731 Sec. IV-B: in the paper's runs the simulation nodes give 12 CPU
 * cores per node to in-situ work).
 *
 * Same definitions as the GPU library and the oracle, independent code:
 *   - per element, the tensor-product transform from GLL nodal values to
 *     Legendre coefficients, sum-factorised (contract i, then j, then k),
 *     each sum started from its first product and accumulated in ascending
 *     index with separately rounded multiply and add (build with
 *     -ffp-contract=off), so the coefficients are the canonical ones;
 *   - norm U2 = sum (J w_k w_j w_i) u^2, energies e = (J g_r g_q g_p) c^2;
 *   - one global value threshold per component: tau = the largest energy v
 *     whose dropped energy S(v) = sum of energies < v stays <= B = tol^2 U2,
 *     every coefficient with e >= tau kept (all ties kept);
 *   - compaction into the blob arrays (bitmap words with bit
 *     f = p + n q + n^2 r, per-element offsets, kept values in element then
 *     f order), inverse of the kept set, error check and the rounding repair
 *     B <- B (tol/rel)^2 (1 - 2^-20), at most 4 times.
 * What differs: the sums are ordinary FP64 sums per thread with Neumaier
 * compensation, merged in thread order, instead of correctly rounded exact
 * sums -- relative error far below 1e-12 -- and the threshold comes from an
 * exponent histogram plus a sort of the boundary bin's energies.
 *
 * Not part of the GPU library: bench.py times it beside the oracle.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double U2, B, tau, dropped, err2, rel;
  uint64_t kept;
  int32_t repair_iters, status;
} cpu_comp_stats;

typedef struct {
  double s, c;  /* Neumaier: running sum and compensation */
} csum;

static inline void cs_add(csum* a, double x) {
  const double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static inline double cs_val(const csum* a) { return a->s + a->c; }

/* y[a] = sum_b M[a][b] x[b*xs], b ascending, no FMA */
static inline double dot_fixed(const double* M, const double* x, int n, int xs) {
  double acc = M[0] * x[0];
  for (int b = 1; b < n; ++b) acc = acc + M[b] * x[b * xs];
  return acc;
}

/* nodal u[k][j][i] -> coefficients c[r][q][p] with matrix A (or inverse with V:
   same three contractions on the other side) */
static void forward_elem(const double* u, const double* A, int n, double* t1, double* t2, double* c) {
  const int n2 = n * n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int p = 0; p < n; ++p) t1[(k * n + j) * n + p] = dot_fixed(A + p * n, u + (k * n + j) * n, n, 1);
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < n; ++p) t2[(k * n + q) * n + p] = dot_fixed(A + q * n, t1 + k * n2 + p, n, n);
  for (int r = 0; r < n; ++r)
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < n; ++p) c[(r * n + q) * n + p] = dot_fixed(A + r * n, t2 + q * n + p, n, n2);
}

static void inverse_elem(const double* c, const double* V, int n, double* s1, double* s2, double* u) {
  const int n2 = n * n;
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < n; ++p) s1[(k * n + q) * n + p] = dot_fixed(V + k * n, c + q * n + p, n, n2);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int p = 0; p < n; ++p) s2[(k * n + j) * n + p] = dot_fixed(V + j * n, s1 + k * n2 + p, n, n);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) u[(k * n + j) * n + i] = dot_fixed(V + i * n, s2 + (k * n + j) * n, n, 1);
}

static inline int ebin(double e) {
  uint64_t b;
  memcpy(&b, &e, 8);
  return (int)((b >> 52) & 2047);
}

static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

#define NB 2048

/* energies of bin b (biased exponent) gathered into v[0..m) */
static void gather_bin(const double* coef, const double* g3, const double* jac, int64_t E, int n3, int b, double* v) {
  uint64_t fill = 0;
#pragma omp parallel
  {
    const int nt = omp_get_num_threads(), t = omp_get_thread_num();
    const int64_t e0 = E * t / nt, e1 = E * (t + 1) / nt;
    uint64_t mine = 0;
    for (int64_t e = e0; e < e1; ++e) {
      const double J = jac ? jac[e] : 1.0;
      for (int f = 0; f < n3; ++f) {
        const double c = coef[e * n3 + f], en = (J * g3[f]) * (c * c);
        mine += ebin(en) == b;
      }
    }
    uint64_t at;
#pragma omp atomic capture
    {
      at = fill;
      fill += mine;
    }
    for (int64_t e = e0; e < e1; ++e) {
      const double J = jac ? jac[e] : 1.0;
      for (int f = 0; f < n3; ++f) {
        const double c = coef[e * n3 + f], en = (J * g3[f]) * (c * c);
        if (ebin(en) == b) v[at++] = en;
      }
    }
  }
}

/* Threshold from the merged exponent histogram: whole bins are dropped while
   the running sum stays within B; the first bin that does not fit is
   gathered and sorted, and its groups of equal values are dropped one by
   one.  tau = the first group (or bin) that no longer fits; +inf when
   everything fits.  Returns -2 when out of memory. */
static int select_tau(const double* coef, const double* g3, const double* jac, int64_t E, int n3, const uint64_t* cnt,
                      const double* bsum, double B, double* tau_out, double* S_out) {
  csum cum = {0, 0};
  for (int b = 0; b < NB; ++b) {
    if (!cnt[b]) continue;
    if (cs_val(&cum) + bsum[b] <= B) {
      cs_add(&cum, bsum[b]);
      continue;
    }
    const uint64_t m = cnt[b];
    double* v = (double*)malloc(m * sizeof(double));
    if (!v) return -2;
    gather_bin(coef, g3, jac, E, n3, b, v);
    qsort(v, m, sizeof(double), cmp_double);
    for (uint64_t i = 0; i < m;) {
      uint64_t k = i;
      csum g = {0, 0};
      while (k < m && v[k] == v[i]) cs_add(&g, v[k++]);
      if (cs_val(&cum) + cs_val(&g) > B) {
        *tau_out = v[i];
        *S_out = cs_val(&cum);
        free(v);
        return 0;
      }
      cs_add(&cum, cs_val(&g));
      i = k;
    }
    free(v);  /* the whole bin fit after all (rounding of its total): go on */
  }
  *tau_out = INFINITY;
  *S_out = cs_val(&cum);
  return 0;
}

/* Compress u (ncomp components, component c at u + c * comp_stride, layout
 * [E][k][j][i]) of order N at relative tolerance tol (tol < 0: keep all).
 * Tables: A[p*n+i], V[i*n+k], w3[n^3], g3[n^3] (FP64).  jac: n_elem
 * Jacobians or NULL.  Outputs: bitmap [ncomp][E][W] words, elem_ptr
 * [ncomp][E+1], values (capacity values_cap doubles; component after
 * component), st[ncomp].  nthreads > 0 sets the OpenMP thread count.
 * Returns 0, -1 on bad arguments or a short value buffer, -2 when out of
 * memory, -4 when the bound is not met after the repairs. */
int isr_cpu_compress(const double* u, int64_t E, int N, int ncomp, int64_t comp_stride, double tol, const double* A,
                     const double* V, const double* w3, const double* g3, const double* jac, int nthreads,
                     uint64_t* bitmap, uint64_t* elem_ptr, double* values, uint64_t values_cap, cpu_comp_stats* st) {
  if (!u || E < 1 || N < 1 || N > 15 || ncomp < 1 || !A || !V || !w3 || !g3 || !bitmap || !elem_ptr || !values || !st)
    return -1;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const int n = N + 1, n3 = n * n * n, W = (n3 + 63) / 64;
  if (comp_stride == 0) comp_stride = E * n3;
  double* coef = (double*)malloc((size_t)E * n3 * sizeof(double));
  uint64_t* ecnt = (uint64_t*)malloc((size_t)E * sizeof(uint64_t));
  const int maxt = omp_get_max_threads();
  uint64_t* tcnt = (uint64_t*)calloc((size_t)maxt * NB, sizeof(uint64_t));
  csum* tsum = (csum*)calloc((size_t)maxt * NB, sizeof(csum));
  csum* tnorm = (csum*)calloc((size_t)maxt * 8, sizeof(csum));  /* padded per thread */
  uint64_t* tkept = (uint64_t*)calloc((size_t)maxt * 8, sizeof(uint64_t));
  if (!coef || !ecnt || !tcnt || !tsum || !tnorm || !tkept) {
    free(coef), free(ecnt), free(tcnt), free(tsum), free(tnorm), free(tkept);
    return -2;
  }
  int rc = 0, etol = 0;
  uint64_t voff = 0;
  for (int comp = 0; comp < ncomp && rc == 0; ++comp) {
    const double* uc = u + comp * comp_stride;
    memset(tcnt, 0, (size_t)maxt * NB * sizeof(uint64_t));
    memset(tsum, 0, (size_t)maxt * NB * sizeof(csum));
    memset(tnorm, 0, (size_t)maxt * 8 * sizeof(csum));
    /* pass 1: transform, norm, energy histogram */
#pragma omp parallel
    {
      const int t = omp_get_thread_num();
      double t1[4096], t2[4096];
      uint64_t* hc = tcnt + (size_t)t * NB;
      csum* hs = tsum + (size_t)t * NB;
      csum* nrm = tnorm + (size_t)t * 8;
#pragma omp for schedule(static)
      for (int64_t e = 0; e < E; ++e) {
        const double J = jac ? jac[e] : 1.0;
        const double* ue = uc + e * n3;
        double* ce = coef + e * n3;
        forward_elem(ue, A, n, t1, t2, ce);
        for (int f = 0; f < n3; ++f) {
          cs_add(nrm, (J * w3[f]) * (ue[f] * ue[f]));
          const double en = (J * g3[f]) * (ce[f] * ce[f]);
          const int b = ebin(en);
          hc[b]++;
          cs_add(&hs[b], en);
        }
      }
    }
    uint64_t cnt[NB];
    double bsum[NB];
    csum U2s = {0, 0};
    for (int b = 0; b < NB; ++b) {
      csum s = {0, 0};
      cnt[b] = 0;
      for (int t = 0; t < maxt; ++t) {
        cnt[b] += tcnt[(size_t)t * NB + b];
        cs_add(&s, cs_val(&tsum[(size_t)t * NB + b]));
      }
      bsum[b] = cs_val(&s);
    }
    for (int t = 0; t < maxt; ++t) cs_add(&U2s, cs_val(&tnorm[(size_t)t * 8]));
    const double U2 = cs_val(&U2s);
    double B = tol < 0 ? 0.0 : (tol * tol) * U2;
    int iters = 0;
    cpu_comp_stats s;
    memset(&s, 0, sizeof(s));
    for (;;) {
      double tau = 0.0, S = 0.0;
      if (tol >= 0 && select_tau(coef, g3, jac, E, n3, cnt, bsum, B, &tau, &S)) {
        rc = -2;
        break;
      }
      /* pass 2: keep flags, per-element counts */
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < E; ++e) {
        const double J = jac ? jac[e] : 1.0;
        uint64_t k = 0;
        for (int f = 0; f < n3; ++f) {
          const double c = coef[e * n3 + f];
          k += ((J * g3[f]) * (c * c)) >= tau;
        }
        ecnt[e] = k;
      }
      /* offsets: per-thread block sums, then a scan */
      uint64_t* ep = elem_ptr + (size_t)comp * (E + 1);
      memset(tkept, 0, (size_t)maxt * 8 * sizeof(uint64_t));
#pragma omp parallel
      {
        const int nt = omp_get_num_threads(), t = omp_get_thread_num();
        const int64_t e0 = E * t / nt, e1 = E * (t + 1) / nt;
        uint64_t a = 0;
        for (int64_t e = e0; e < e1; ++e) a += ecnt[e];
        tkept[(size_t)t * 8] = a;
#pragma omp barrier
#pragma omp single
        {
          uint64_t run = 0;
          for (int q = 0; q < nt; ++q) {
            const uint64_t x = tkept[(size_t)q * 8];
            tkept[(size_t)q * 8] = run;
            run += x;
          }
        }
        uint64_t run = tkept[(size_t)t * 8];
        for (int64_t e = e0; e < e1; ++e) {
          ep[e] = run;
          run += ecnt[e];
        }
        if (t == nt - 1) ep[E] = run;
      }
      const uint64_t kept = ep[E];
      if (voff + kept > values_cap) {
        rc = -1;
        break;
      }
      /* pass 3: bitmap, values, inverse of the kept set, error */
      memset(tnorm, 0, (size_t)maxt * 8 * sizeof(csum));
#pragma omp parallel
      {
        const int t = omp_get_thread_num();
        double m[4096], s1[4096], s2[4096], rec[4096];
        csum* err = tnorm + (size_t)t * 8;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
          const double J = jac ? jac[e] : 1.0;
          const double* ce = coef + e * n3;
          uint64_t* bw = bitmap + ((size_t)comp * E + e) * W;
          for (int w = 0; w < W; ++w) bw[w] = 0;
          uint64_t pos = voff + ep[e];
          for (int f = 0; f < n3; ++f) {
            const double c = ce[f];
            const int keep = ((J * g3[f]) * (c * c)) >= tau;
            m[f] = keep ? c : 0.0;
            if (keep) {
              bw[f >> 6] |= 1ull << (f & 63);
              values[pos++] = c;
            }
          }
          inverse_elem(m, V, n, s1, s2, rec);
          const double* ue = uc + e * n3;
          for (int f = 0; f < n3; ++f) {
            const double d = ue[f] - rec[f];
            cs_add(err, (J * w3[f]) * (d * d));
          }
        }
      }
      csum e2 = {0, 0};
      for (int t = 0; t < maxt; ++t) cs_add(&e2, cs_val(&tnorm[(size_t)t * 8]));
      const double err2 = cs_val(&e2);
      const double rel = U2 > 0 ? sqrt(err2 / U2) : 0.0;
      s.U2 = U2;
      s.B = B;
      s.tau = tau;
      s.dropped = S;
      s.err2 = err2;
      s.rel = rel;
      s.kept = kept;
      s.repair_iters = iters;
      if (tol < 0 || rel <= tol || iters >= 4) break;
      const double fr = tol / rel;
      B = (B * (fr * fr)) * (1.0 - 0x1p-20);
      ++iters;
    }
    if (rc) break;
    s.status = (tol >= 0 && s.rel > tol) ? -4 : 0;
    st[comp] = s;
    voff += s.kept;
    if (s.status) etol = 1;
  }
  free(coef), free(ecnt), free(tcnt), free(tsum), free(tnorm), free(tkept);
  return rc ? rc : (etol ? -4 : 0);
}
