/*
 * Plain FP64 string-basis sigma = H c for the oracle (test infrastructure only).
 *
 * The paper's problem statement (Results, "SBCI1 algorithm") is the
 * Hamiltonian in a Slater-determinant basis; this file evaluates sigma row by
 * row from the Slater-Condon rules, with no blocking, no GEMM and no
 * intermediate beyond what the rules need:
 *
 *   sigma[I] = D[I] c[I]
 *            + sum over alpha singles q->p of I:  s * (h_pq + sum_{r in Ia\q}((pq|rr)-(pr|rq))
 *                                                       + sum_{r in Ib} (pq|rr)) * c[J]
 *            + the same for beta singles
 *            + sum over alpha doubles (q1<q2 -> p1<p2): s * ((p1q1|p2q2)-(p1q2|p2q1)) * c[J]
 *            + the same for beta doubles
 *            + sum over alpha single x beta single:     sa * sb * (pq|rs) * c[J]
 *
 * Strings: m-subsets of {0..N-1} as bit masks, ascending; rank via the
 * combinatorial number system.  Determinant index = Ia * Nb + Ib.
 * Sign of E_pq|I>: (-1)^(occupied orbitals strictly between p and q).
 *
 * Entry points (plain C ABI, all host pointers):
 *   oracle_sigma(norb, na, nb, h1[N*N], eri[N^4], c[ndet], out[ndet])
 *   oracle_sigma_rows(norb, na, nb, h1, eri, c, rows[nrows], nrows, out[nrows])
 * Parallelised over rows with OpenMP only.
 *
 * Each string's own excitations (its singles q->p with target and sign, its
 * doubles with target and sign times the integral difference) are listed
 * once at setup, in the loop order of the rules above; a row then walks
 * those lists.  Every term and the order of the sums are those of the plain
 * per-row loops, so sigma is the same to the last bit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* one single excitation q -> p of a string: target string j, sign */
typedef struct {
  int p, q;
  int64_t j;
  double sg;
} sgl_t;

/* one same-spin double of a string: target j, sign * ((p1q1|p2q2) - (p1q2|p2q1)) */
typedef struct {
  int64_t j;
  double w;
} dbl_t;

typedef struct {
  int norb, na, nb;
  int64_t nsa, nsb;
  uint64_t *sa, *sb;
  int64_t binom[65][65];
  const double *h, *g;
  int ns1[2], nd2[2];      /* singles / doubles per string of each spin       */
  sgl_t *s1[2];            /* [nstrings][ns1] per spin                        */
  dbl_t *d2[2];            /* [nstrings][nd2] per spin                        */
} sys_t;

static int64_t choose(int n, int k) {
  /* Pascal's triangle: exact for n <= 64 */
  static int64_t t[65][65];
  static int ready = 0;
  if (!ready) {
    for (int i = 0; i <= 64; ++i) {
      t[i][0] = 1;
      for (int j = 1; j <= 64; ++j) t[i][j] = (i == 0) ? 0 : t[i - 1][j - 1] + t[i - 1][j];
    }
    ready = 1;
  }
  if (n < 0 || k < 0 || k > n || n > 64) return 0;
  return t[n][k];
}

static uint64_t *enum_strings(int n, int m, int64_t *count) {
  int64_t cnt = choose(n, m);
  uint64_t *out = (uint64_t *)malloc(sizeof(uint64_t) * (cnt > 0 ? cnt : 1));
  if (m == 0) { out[0] = 0; *count = 1; return out; }
  /* next bit permutation yields masks in ascending order */
  uint64_t v = (m == 64) ? ~0ull : ((1ull << m) - 1);
  for (int64_t i = 0; i < cnt; ++i) {
    out[i] = v;
    uint64_t t = v | (v - 1);
    uint64_t w = (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctzll(v) + 1));
    v = w;
  }
  *count = cnt;
  return out;
}

static int64_t rank_of(const sys_t *S, uint64_t mask) {
  int64_t r = 0;
  int k = 1;
  while (mask) {
    int o = __builtin_ctzll(mask);
    r += S->binom[o][k];
    ++k;
    mask &= mask - 1;
  }
  return r;
}

static inline double G(const sys_t *S, int p, int q, int r, int s) {
  int n = S->norb;
  return S->g[((p * n + q) * n + r) * n + s];
}

static inline int between_parity(uint64_t mask, int a, int b) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  uint64_t m = (hi >= 64 ? ~0ull : ((1ull << hi) - 1)) & ~((lo + 1 >= 64) ? ~0ull : ((1ull << (lo + 1)) - 1));
  return __builtin_popcountll(mask & m) & 1;
}

static double diag_elem(const sys_t *S, uint64_t ma, uint64_t mb) {
  int n = S->norb;
  double e = 0.0;
  for (int p = 0; p < n; ++p) {
    int pa = (ma >> p) & 1, pb = (mb >> p) & 1;
    if (pa) e += S->h[p * n + p];
    if (pb) e += S->h[p * n + p];
    for (int q = 0; q < n; ++q) {
      int qa = (ma >> q) & 1, qb = (mb >> q) & 1;
      double J = G(S, p, p, q, q), K = G(S, p, q, q, p);
      if (pa && qa) e += 0.5 * (J - K);
      if (pb && qb) e += 0.5 * (J - K);
      if (pa && qb) e += J;
    }
  }
  return e;
}

/* the excitation lists of one string (mask m of spin sp) */
static void list_string(const sys_t *S, uint64_t m, sgl_t *s1, dbl_t *d2) {
  const int n = S->norb;
  int k = 0;
  for (int q = 0; q < n; ++q) {
    if (!((m >> q) & 1)) continue;
    for (int p = 0; p < n; ++p) {
      if ((m >> p) & 1) continue;
      uint64_t nm = (m & ~(1ull << q)) | (1ull << p);
      s1[k].p = p;
      s1[k].q = q;
      s1[k].sg = between_parity(m, p, q) ? -1.0 : 1.0;
      s1[k].j = rank_of(S, nm);
      ++k;
    }
  }
  k = 0;
  for (int q1 = 0; q1 < n; ++q1) {
    if (!((m >> q1) & 1)) continue;
    for (int q2 = q1 + 1; q2 < n; ++q2) {
      if (!((m >> q2) & 1)) continue;
      for (int p1 = 0; p1 < n; ++p1) {
        if ((m >> p1) & 1) continue;
        for (int p2 = p1 + 1; p2 < n; ++p2) {
          if ((m >> p2) & 1) continue;
          double v = G(S, p1, q1, p2, q2) - G(S, p1, q2, p2, q1);
          uint64_t m1 = (m & ~(1ull << q2)) | (1ull << p2);
          int t1 = between_parity(m, p2, q2);
          uint64_t m2 = (m1 & ~(1ull << q1)) | (1ull << p1);
          int t2 = between_parity(m1, p1, q1);
          double sg = (t1 ^ t2) ? -1.0 : 1.0;
          d2[k].j = rank_of(S, m2);
          d2[k].w = sg * v;
          ++k;
        }
      }
    }
  }
}

/* sigma for one determinant row (ia, ib) */
static double row_sigma(const sys_t *S, int64_t ia, int64_t ib, const double *c) {
  const int n = S->norb;
  const int64_t nsb = S->nsb;
  const uint64_t ma = S->sa[ia], mb = S->sb[ib];
  double acc = diag_elem(S, ma, mb) * c[ia * nsb + ib];

  for (int spin = 0; spin < 2; ++spin) {
    const uint64_t m = spin == 0 ? ma : mb;
    const uint64_t mo = spin == 0 ? mb : ma;
    const int64_t is = spin == 0 ? ia : ib;
    /* singles q -> p */
    const sgl_t *e1 = S->s1[spin] + is * S->ns1[spin];
    for (int e = 0; e < S->ns1[spin]; ++e) {
      const int p = e1[e].p, q = e1[e].q;
      double v = S->h[p * n + q];
      for (int r = 0; r < n; ++r) {
        if (r != q && ((m >> r) & 1)) v += G(S, p, q, r, r) - G(S, p, r, r, q);
        if ((mo >> r) & 1) v += G(S, p, q, r, r);
      }
      int64_t idx = spin == 0 ? e1[e].j * nsb + ib : ia * nsb + e1[e].j;
      acc += e1[e].sg * v * c[idx];
    }
    /* same-spin doubles */
    const dbl_t *e2 = S->d2[spin] + is * S->nd2[spin];
    for (int e = 0; e < S->nd2[spin]; ++e) {
      int64_t idx = spin == 0 ? e2[e].j * nsb + ib : ia * nsb + e2[e].j;
      acc += e2[e].w * c[idx];
    }
  }
  /* opposite-spin doubles: alpha q->p, beta s->r */
  const sgl_t *ea = S->s1[0] + ia * S->ns1[0];
  const sgl_t *eb = S->s1[1] + ib * S->ns1[1];
  for (int a = 0; a < S->ns1[0]; ++a) {
    const int p = ea[a].p, q = ea[a].q;
    const double sa = ea[a].sg;
    const int64_t ja = ea[a].j;
    for (int b = 0; b < S->ns1[1]; ++b)
      acc += sa * eb[b].sg * G(S, p, q, eb[b].p, eb[b].q) * c[ja * nsb + eb[b].j];
  }
  return acc;
}

static int setup(sys_t *S, int norb, int na, int nb, const double *h1, const double *eri) {
  memset(S, 0, sizeof(*S));
  if (norb < 1 || norb > 63 || na < 0 || nb < 0 || na > norb || nb > norb) return -1;
  S->norb = norb; S->na = na; S->nb = nb; S->h = h1; S->g = eri;
  for (int i = 0; i <= 64; ++i)
    for (int k = 0; k <= 64; ++k) S->binom[i][k] = choose(i, k);
  S->sa = enum_strings(norb, na, &S->nsa);
  S->sb = enum_strings(norb, nb, &S->nsb);
  for (int sp = 0; sp < 2; ++sp) {
    const int m = sp == 0 ? na : nb;
    const int64_t ns = sp == 0 ? S->nsa : S->nsb;
    const uint64_t *str = sp == 0 ? S->sa : S->sb;
    S->ns1[sp] = m * (norb - m);
    S->nd2[sp] = (int)(choose(m, 2) * choose(norb - m, 2));
    S->s1[sp] = (sgl_t *)malloc(sizeof(sgl_t) * (size_t)(ns * S->ns1[sp] + 1));
    S->d2[sp] = (dbl_t *)malloc(sizeof(dbl_t) * (size_t)(ns * S->nd2[sp] + 1));
    if (!S->s1[sp] || !S->d2[sp]) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ns; ++i)
      list_string(S, str[i], S->s1[sp] + i * S->ns1[sp], S->d2[sp] + i * S->nd2[sp]);
  }
  return 0;
}

static void teardown(sys_t *S) {
  free(S->sa);
  free(S->sb);
  for (int sp = 0; sp < 2; ++sp) {
    free(S->s1[sp]);
    free(S->d2[sp]);
  }
}

int oracle_sigma(int norb, int na, int nb, const double *h1, const double *eri,
                 const double *c, double *out) {
  sys_t S;
  const int rc = setup(&S, norb, na, nb, h1, eri);
  if (rc) {
    if (rc == -2) teardown(&S);
    return rc;
  }
  const int64_t nsa = S.nsa, nsb = S.nsb;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ia = 0; ia < nsa; ++ia)
    for (int64_t ib = 0; ib < nsb; ++ib) out[ia * nsb + ib] = row_sigma(&S, ia, ib, c);
  teardown(&S);
  return 0;
}

int oracle_sigma_rows(int norb, int na, int nb, const double *h1, const double *eri,
                      const double *c, const int64_t *rows, int64_t nrows, double *out) {
  sys_t S;
  const int rc = setup(&S, norb, na, nb, h1, eri);
  if (rc) {
    if (rc == -2) teardown(&S);
    return rc;
  }
  const int64_t nsb = S.nsb;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nrows; ++i) out[i] = row_sigma(&S, rows[i] / nsb, rows[i] % nsb, c);
  teardown(&S);
  return 0;
}

int oracle_hdiag(int norb, int na, int nb, const double *h1, const double *eri, double *out) {
  sys_t S;
  const int rc = setup(&S, norb, na, nb, h1, eri);
  if (rc) {
    if (rc == -2) teardown(&S);
    return rc;
  }
  const int64_t nsa = S.nsa, nsb = S.nsb;
#pragma omp parallel for schedule(static)
  for (int64_t ia = 0; ia < nsa; ++ia)
    for (int64_t ib = 0; ib < nsb; ++ib) out[ia * nsb + ib] = diag_elem(&S, S.sa[ia], S.sb[ib]);
  teardown(&S);
  return 0;
}
