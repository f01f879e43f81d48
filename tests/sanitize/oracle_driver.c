/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built
 * with gcc by tests/test_sanitizers.py): forward, VJP, Jacobian, final state
 * and uncompute on layered and random circuits with every gate type, Z and
 * general Pauli observables, one and several threads, both parallel modes;
 * invalid gate lists must be rejected.  Checks only what holds for any
 * correct run (finite values, |<O>| <= 1, unit norm, the Jacobian contracted
 * with G equals the VJP); the numerical pins are in test_oracle_pins.py.
 * Exit status 0 when every check holds; a sanitizer report aborts. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int qtm_oracle_forward(int, const int32_t *, int, int, int, const uint64_t *, const uint64_t *, int, int,
                       const double *, const double *, double *, int, int);
int qtm_oracle_vjp(int, const int32_t *, int, int, int, const uint64_t *, const uint64_t *, int, int,
                   const double *, const double *, const double *, double *, double *, double *, double *,
                   int, int);
int qtm_oracle_jacobian(int, const int32_t *, int, int, int, const uint64_t *, const uint64_t *, int, int,
                        const double *, const double *, double *, double *, double *, int, int);
int qtm_oracle_state(int, const int32_t *, int, int, int, const double *, const double *, double *);
int qtm_oracle_uncompute(int, const int32_t *, int, int, int, const double *, const double *, double *);

static int g_fail = 0;
static void check(int ok, const char *what, int k) {
  if (!ok) {
    fprintf(stderr, "FAIL: %s (case %d)\n", what, k);
    ++g_fail;
  }
}

static uint64_t rs = 88172645463325252ull;
static uint64_t rnd(void) {
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return rs;
}
static double unif(double a, double b) { return a + (b - a) * (double)(rnd() >> 11) / 9007199254740992.0; }

/* case k: layered RX/RY/RZ + CNOT ring (k even) or a random mix of every gate type */
static int make(int k, int n, int32_t *g, int *ni, int *nw) {
  int c = 0;
  if (k % 2 == 0) {
    const int L = 2;
    for (int l = 0; l < L; ++l) {
      for (int q = 0; q < n; ++q) { int32_t r[5] = {0, q, 0, 1, q}; for (int i = 0; i < 5; ++i) g[5 * c + i] = r[i]; ++c; }
      for (int q = 0; q < n; ++q) { int32_t r[5] = {1, q, 0, 2, l * 2 * n + q}; for (int i = 0; i < 5; ++i) g[5 * c + i] = r[i]; ++c; }
      for (int q = 0; q < n; ++q) { int32_t r[5] = {2, q, 0, 2, l * 2 * n + n + q}; for (int i = 0; i < 5; ++i) g[5 * c + i] = r[i]; ++c; }
      for (int q = 0; q < n && n > 1; ++q) { int32_t r[5] = {3, q, (q + 1) % n, 0, 0}; for (int i = 0; i < 5; ++i) g[5 * c + i] = r[i]; ++c; }
    }
    *ni = n;
    *nw = 2 * n * L;
    return c;
  }
  for (int j = 0; j < 40; ++j) {
    const int r = (int)(rnd() % 12), q = (int)(rnd() % n);
    int q1 = (int)(rnd() % n);
    if (n > 1) while (q1 == q) q1 = (int)(rnd() % n);
    int32_t *e = g + 5 * c;
    if (r < 4) {
      const int src = 1 + (int)(rnd() % 3);
      e[0] = (int)(rnd() % 3); e[1] = q; e[2] = src == 3 ? (int)(rnd() % 5) : 0; e[3] = src;
      e[4] = (int)(rnd() % (src == 2 ? 5 : 4));
    } else if (r < 7) {
      e[0] = 5 + (int)(rnd() % 9); e[1] = q; e[2] = 0; e[3] = 0; e[4] = 0;
    } else if (n > 1 && r < 10) {
      e[0] = r < 9 ? 3 : 4; e[1] = q; e[2] = q1; e[3] = 0; e[4] = 0;
    } else if (n > 1) {
      e[0] = 14 + (int)(rnd() % 3); e[1] = q; e[2] = q1; e[3] = 1 + (int)(rnd() % 2); e[4] = (int)(rnd() % 4);
    } else {
      continue;
    }
    ++c;
  }
  *ni = 4;
  *nw = 5;
  return c;
}

int main(void) {
  enum { MAXG = 400, B = 5 };
  int32_t g[5 * MAXG];
  for (int k = 0; k < 16; ++k) {
    const int n = 1 + k % 7;
    int ni = 0, nw = 0;
    const int ng = make(k, n, g, &ni, &nw);
    const int M = 3;
    uint64_t zm[3], xm[3];
    const uint64_t all = ((uint64_t)1 << n) - 1;
    for (int m = 0; m < M; ++m) {
      zm[m] = (m == 0 ? 1u : rnd()) & all;
      xm[m] = (k % 4 == 1) ? (rnd() & all) : 0;
    }
    const uint64_t *xp = (k % 4 == 1) ? xm : NULL;
    double *x = malloc(sizeof(double) * B * ni), *w = malloc(sizeof(double) * nw);
    double *G = malloc(sizeof(double) * B * M), *ev = malloc(sizeof(double) * B * M);
    double *gw = malloc(sizeof(double) * nw), *gx = malloc(sizeof(double) * B * ni);
    double *go = malloc(sizeof(double) * B * ng);
    double *jw = malloc(sizeof(double) * B * M * nw), *jx = malloc(sizeof(double) * B * M * ni);
    double *ev2 = malloc(sizeof(double) * B * M), *st = malloc(sizeof(double) * 2 * ((size_t)1 << n));
    for (int i = 0; i < B * ni; ++i) x[i] = unif(-3.14159265358979323846, 3.14159265358979323846);
    for (int i = 0; i < nw; ++i) w[i] = unif(-3.14159265358979323846, 3.14159265358979323846);
    for (int i = 0; i < B * M; ++i) G[i] = unif(-1, 1);
    for (int par = 0; par < 2; ++par)
      for (int th = 1; th <= 3; th += 2) {
        check(qtm_oracle_forward(n, g, ng, ni, nw, zm, xp, M, B, x, w, ev, th, par) == 0, "forward", k);
        for (int i = 0; i < B * M; ++i) check(isfinite(ev[i]) && fabs(ev[i]) <= 1 + 1e-12, "|<O>| <= 1", k);
        check(qtm_oracle_vjp(n, g, ng, ni, nw, zm, xp, M, B, x, w, G, ev2, gw, gx, go, th, par) == 0, "vjp", k);
        for (int i = 0; i < B * M; ++i) check(fabs(ev2[i] - ev[i]) <= 1e-13, "vjp expvals", k);
        check(qtm_oracle_jacobian(n, g, ng, ni, nw, zm, xp, M, B, x, w, NULL, jw, jx, th, par) == 0, "jacobian", k);
        for (int j = 0; j < nw; ++j) {
          double s = 0;
          for (int b = 0; b < B; ++b)
            for (int m = 0; m < M; ++m) s += G[b * M + m] * jw[((size_t)b * M + m) * nw + j];
          check(fabs(s - gw[j]) <= 1e-10, "J_w contracted = VJP", k);
        }
        for (int b = 0; b < B; ++b)
          for (int i = 0; i < ni; ++i) {
            double s = 0;
            for (int m = 0; m < M; ++m) s += G[b * M + m] * jx[((size_t)b * M + m) * ni + i];
            check(fabs(s - gx[b * ni + i]) <= 1e-10, "J_x contracted = VJP", k);
          }
      }
    check(qtm_oracle_state(n, g, ng, ni, nw, x, w, st) == 0, "state", k);
    double nr = 0;
    for (size_t i = 0; i < 2 * ((size_t)1 << n); ++i) nr += st[i] * st[i];
    check(fabs(nr - 1) <= 1e-12, "unit norm", k);
    double a0 = 0;
    check(qtm_oracle_uncompute(n, g, ng, ni, nw, x, w, &a0) == 0 && fabs(a0 - 1) <= 1e-10, "uncompute", k);
    /* invalid: qubit out of range, then an unknown gate type */
    if (ng > 0) {
      const int32_t keep = g[1];
      g[1] = n;
      check(qtm_oracle_forward(n, g, ng, ni, nw, zm, xp, M, B, x, w, ev, 1, 0) != 0, "reject bad qubit", k);
      g[1] = keep;
      const int32_t kt = g[0];
      g[0] = 99;
      check(qtm_oracle_forward(n, g, ng, ni, nw, zm, xp, M, B, x, w, ev, 1, 0) != 0, "reject bad type", k);
      g[0] = kt;
    }
    free(x); free(w); free(G); free(ev); free(gw); free(gx); free(go); free(jw); free(jx); free(ev2); free(st);
  }
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("oracle driver ok\n");
  return 0;
}
