/*
 * qtm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statevector simulator in complex128
 * for the layered variational circuits of the paper (Eq. (1)-(7)).  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant with the GPU library: it
 * defines its own copy of the gate-record format and recomputes everything
 * from the definitions.
 *
 * What it computes (paper Sec. II):
 *   - Eq. (1)-(2): <O> = <0| U^dag O U |0>, U = G_N ... G_1 applied in list
 *     order to |0...0>.
 *   - Eq. (3)-(4): the state is evolved once, then every observable O_m (a
 *     Pauli-Z string, diagonal with entries (-1)^popcount(x & S_m)) is read
 *     from it.
 *   - Eq. (5) and the reverse ("adjoint") gradient the paper cites (Jones and
 *     Gacon, Algorithm 1): run the circuit backwards, un-applying each gate on
 *     the forward state phi, applying the derivative of the gate matrix to
 *     phi to get mu, and taking 2 Re<lambda|mu> with lambda the back-
 *     propagated bra.  Two variants:
 *       * Jacobian: the paper's multi-observable extension, one bra
 *         lambda_m = O_m phi per observable sharing one un-computed phi,
 *         giving the (B, M, |Theta|) result of Sec. II-B;
 *       * VJP: the same sweep with the single bra lambda = sum_m G_m O_m phi.
 *   - Eq. (6): a batch of inputs with shared weights.  Samples are split over
 *     T threads following Sec. II-B: equal shares, the first
 *     B - T*floor(B/T) threads take one more sample.
 *
 * Conventions (readings of points the paper leaves open):
 *   - basis index x = sum_q b_q 2^q (qubit q is bit q);
 *   - RX = [[c, -is], [-is, c]], RY = [[c, -s], [s, c]],
 *     RZ = diag(e^{-i t/2}, e^{i t/2}), c = cos(t/2), s = sin(t/2);
 *   - CNOT(c, t) swaps the amplitudes x and x|2^t for every x with b_c = 1,
 *     b_t = 0;  CZ(a, b) negates every amplitude with b_a = b_b = 1.
 *
 * Gate record: int32 x 5 = type, q0, q1, src, index.
 *   type 0 RX, 1 RY, 2 RZ, 3 CNOT (q0 control, q1 target), 4 CZ;
 *   fixed one-qubit gates on q0: 5 H, 6 X, 7 Y, 8 Z, 9 S, 10 S^dag, 11 T,
 *   12 T^dag, 13 SX (square root of X);
 *   controlled rotations 14 CRX, 15 CRY, 16 CRZ: q0 control, q1 target, the
 *   rotation applied where the control bit is 1 (src 1 or 2 only);
 *   src 1 = inputs[index], 2 = weights[index],
 *   3 = weights[q1] * inputs[index] (trainable input scaling of the
 *       ansatz of Sec. III-A, Eq. (7): angle lambda_j s_i; the chain rule
 *       gives dL/dlambda_j = g s_i and dL/ds_i = g lambda_j for the angle
 *       derivative g).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { O_RX = 0, O_RY = 1, O_RZ = 2, O_CNOT = 3, O_CZ = 4, O_H = 5, O_SX = 13, O_CRX = 14,
       O_CRZ = 16 };
enum { O_SRC_NONE = 0, O_SRC_INPUT = 1, O_SRC_WEIGHT = 2, O_SRC_SCALED = 3 };

/* Observable m is the Pauli string with X-part xmasks[m] and Z-part
 * masks[m]: on qubit q the factor is I (bits 0, 0), X (1, 0), Y (1, 1) or
 * Z (0, 1).  xmasks may be NULL (every observable a Z string). */
typedef struct {
  int n;
  const int32_t *gates;
  int n_gates;
  int n_inputs;
  int n_weights;
  const uint64_t *masks;
  int n_obs;
  const uint64_t *xmasks;
} circ_t;

static uint64_t xmask_of(const circ_t *c, int m) { return c->xmasks ? c->xmasks[m] : 0; }

static int is_rot(int type) { return type == O_RX || type == O_RY || type == O_RZ; }
static int is_crot(int type) { return type >= O_CRX && type <= O_CRZ; }
static int is_fixed(int type) { return type >= O_H && type <= O_SX; }
static int is_param(int type) { return is_rot(type) || is_crot(type); }

static int check_circuit(const circ_t *c) {
  if (c->n < 1 || c->n > 30 || c->n_gates < 0 || c->n_obs < 0) return -1;
  for (int k = 0; k < c->n_gates; ++k) {
    const int32_t *g = c->gates + 5 * k;
    if (g[0] < 0 || g[0] > O_CRZ) return -1;
    if (g[1] < 0 || g[1] >= c->n) return -1;
    if (is_fixed(g[0])) continue;
    if (!is_rot(g[0])) {
      if (g[2] < 0 || g[2] >= c->n || g[2] == g[1]) return -1;
    }
    if (is_crot(g[0]) && g[3] != O_SRC_INPUT && g[3] != O_SRC_WEIGHT) return -1;
    if (is_param(g[0])) {
      if (g[3] == O_SRC_INPUT && (g[4] < 0 || g[4] >= c->n_inputs)) return -1;
      if (g[3] == O_SRC_WEIGHT && (g[4] < 0 || g[4] >= c->n_weights)) return -1;
      if (g[3] == O_SRC_SCALED &&
          (g[4] < 0 || g[4] >= c->n_inputs || g[2] < 0 || g[2] >= c->n_weights))
        return -1;
      if (g[3] != O_SRC_INPUT && g[3] != O_SRC_WEIGHT && g[3] != O_SRC_SCALED) return -1;
    }
  }
  for (int m = 0; m < c->n_obs; ++m)
    if (c->n < 64 && ((c->masks[m] | xmask_of(c, m)) >> c->n) != 0) return -1;
  return 0;
}

static double angle_of(const int32_t *g, const double *x_b, const double *w) {
  if (g[3] == O_SRC_SCALED) return w[g[2]] * x_b[g[4]];
  return g[3] == O_SRC_INPUT ? x_b[g[4]] : w[g[4]];
}

/* Gate matrix of a rotation, from its definition. */
static void rot_matrix(int type, double t, cplx u[2][2]) {
  double c = cos(t / 2), s = sin(t / 2);
  if (type == O_RX) {
    u[0][0] = c;       u[0][1] = -I * s;
    u[1][0] = -I * s;  u[1][1] = c;
  } else if (type == O_RY) {
    u[0][0] = c;  u[0][1] = -s;
    u[1][0] = s;  u[1][1] = c;
  } else {
    u[0][0] = cexp(-I * t / 2);  u[0][1] = 0;
    u[1][0] = 0;                 u[1][1] = cexp(I * t / 2);
  }
}

/* Entrywise derivative d/dt of the rotation matrix above. */
static void rot_deriv(int type, double t, cplx d[2][2]) {
  double c = cos(t / 2), s = sin(t / 2);
  if (type == O_RX) {
    d[0][0] = -s / 2;       d[0][1] = -I * c / 2;
    d[1][0] = -I * c / 2;   d[1][1] = -s / 2;
  } else if (type == O_RY) {
    d[0][0] = -s / 2;  d[0][1] = -c / 2;
    d[1][0] = c / 2;   d[1][1] = -s / 2;
  } else {
    d[0][0] = -I / 2 * cexp(-I * t / 2);  d[0][1] = 0;
    d[1][0] = 0;                          d[1][1] = I / 2 * cexp(I * t / 2);
  }
}

/* Matrices of the fixed one-qubit gates, from their definitions. */
static void fixed_matrix(int type, cplx u[2][2]) {
  const double r = 1.0 / sqrt(2.0);
  u[0][0] = 1; u[0][1] = 0; u[1][0] = 0; u[1][1] = 1;
  switch (type) {
    case 5:  u[0][0] = r; u[0][1] = r; u[1][0] = r; u[1][1] = -r; break;   /* H */
    case 6:  u[0][0] = 0; u[0][1] = 1; u[1][0] = 1; u[1][1] = 0; break;    /* X */
    case 7:  u[0][0] = 0; u[0][1] = -I; u[1][0] = I; u[1][1] = 0; break;   /* Y */
    case 8:  u[1][1] = -1; break;                                         /* Z */
    case 9:  u[1][1] = I; break;                                          /* S */
    case 10: u[1][1] = -I; break;                                         /* S^dag */
    case 11: u[1][1] = (1 + I) * r; break;                                /* T: e^{i pi/4} */
    case 12: u[1][1] = (1 - I) * r; break;                                /* T^dag */
    default:                                                              /* SX */
      u[0][0] = (1 + I) / 2; u[0][1] = (1 - I) / 2;
      u[1][0] = (1 - I) / 2; u[1][1] = (1 + I) / 2;
  }
}

static void dagger(cplx u[2][2], cplx out[2][2]) {
  out[0][0] = conj(u[0][0]); out[0][1] = conj(u[1][0]);
  out[1][0] = conj(u[0][1]); out[1][1] = conj(u[1][1]);
}

/* Apply a 2x2 matrix to qubit q: for every x with b_q = 0 the pair
 * (psi[x], psi[x | 2^q]) is multiplied by u.  par = 1 spreads the loop over
 * OpenMP threads (one large sample); par = 0 runs it on the calling thread. */
static void apply_1q(cplx *psi, int n, int q, cplx u[2][2], int par) {
  const int64_t dim = (int64_t)1 << n, bit = (int64_t)1 << q;
#pragma omp parallel for if (par) schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    if (x & bit) continue;
    cplx a = psi[x], b = psi[x | bit];
    psi[x] = u[0][0] * a + u[0][1] * b;
    psi[x | bit] = u[1][0] * a + u[1][1] * b;
  }
}

/* As apply_1q on qubit q, only where bit ctl is 1 (a controlled gate). */
static void apply_1q_ctl(cplx *psi, int n, int ctl, int q, cplx u[2][2], int par) {
  const int64_t dim = (int64_t)1 << n, bit = (int64_t)1 << q, cb = (int64_t)1 << ctl;
#pragma omp parallel for if (par) schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    if ((x & bit) || !(x & cb)) continue;
    cplx a = psi[x], b = psi[x | bit];
    psi[x] = u[0][0] * a + u[0][1] * b;
    psi[x | bit] = u[1][0] * a + u[1][1] * b;
  }
}

static void apply_cnot(cplx *psi, int n, int ctl, int tgt, int par) {
  const int64_t dim = (int64_t)1 << n, cb = (int64_t)1 << ctl, tb = (int64_t)1 << tgt;
#pragma omp parallel for if (par) schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    if ((x & cb) && !(x & tb)) {
      cplx t = psi[x];
      psi[x] = psi[x | tb];
      psi[x | tb] = t;
    }
  }
}

static void apply_cz(cplx *psi, int n, int a, int b, int par) {
  const int64_t dim = (int64_t)1 << n, ab = (int64_t)1 << a, bb = (int64_t)1 << b;
#pragma omp parallel for if (par) schedule(static)
  for (int64_t x = 0; x < dim; ++x)
    if ((x & ab) && (x & bb)) psi[x] = -psi[x];
}

/* Apply gate k (inverse = 1 applies its adjoint). */
static void apply_gate(cplx *psi, int n, const int32_t *g, const double *x_b,
                       const double *w, int inverse, int par) {
  if (is_rot(g[0]) || is_fixed(g[0])) {
    cplx u[2][2], ud[2][2];
    if (is_rot(g[0])) rot_matrix(g[0], angle_of(g, x_b, w), u);
    else fixed_matrix(g[0], u);
    if (inverse) {
      dagger(u, ud);
      apply_1q(psi, n, g[1], ud, par);
    } else {
      apply_1q(psi, n, g[1], u, par);
    }
  } else if (is_crot(g[0])) {
    cplx u[2][2], ud[2][2];
    rot_matrix(g[0] - O_CRX, angle_of(g, x_b, w), u);
    if (inverse) {
      dagger(u, ud);
      apply_1q_ctl(psi, n, g[1], g[2], ud, par);
    } else {
      apply_1q_ctl(psi, n, g[1], g[2], u, par);
    }
  } else if (g[0] == O_CNOT) {
    apply_cnot(psi, n, g[1], g[2], par); /* self-inverse */
  } else {
    apply_cz(psi, n, g[1], g[2], par); /* self-inverse */
  }
}

/* |psi> = U |0...0> (Eq. (4)). */
static void evolve(const circ_t *c, const double *x_b, const double *w, cplx *psi, int par) {
  const int64_t dim = (int64_t)1 << c->n;
  memset(psi, 0, sizeof(cplx) * dim);
  psi[0] = 1.0;
  for (int k = 0; k < c->n_gates; ++k)
    apply_gate(psi, c->n, c->gates + 5 * k, x_b, w, 0, par);
}

static double zsign(int64_t x, uint64_t mask) {
  return (__builtin_popcountll((uint64_t)x & mask) & 1) ? -1.0 : 1.0;
}

/* v <- P v for the Pauli string (xm, zm): the tensor product of one Pauli
 * matrix per qubit, X = [[0, 1], [1, 0]], Y = [[0, -i], [i, 0]],
 * Z = [[1, 0], [0, -1]], each applied as a one-qubit gate. */
static void apply_pauli(cplx *v, int n, uint64_t xm, uint64_t zm, int par) {
  for (int q = 0; q < n; ++q) {
    const int xb = (int)((xm >> q) & 1), zb = (int)((zm >> q) & 1);
    if (!xb && !zb) continue;
    cplx u[2][2];
    if (xb && zb) {
      u[0][0] = 0;  u[0][1] = -I;
      u[1][0] = I;  u[1][1] = 0;
    } else if (xb) {
      u[0][0] = 0;  u[0][1] = 1;
      u[1][0] = 1;  u[1][1] = 0;
    } else {
      u[0][0] = 1;  u[0][1] = 0;
      u[1][0] = 0;  u[1][1] = -1;
    }
    apply_1q(v, n, q, u, par);
  }
}

/* <psi|O_m|psi> for every observable (Eq. (3)).  A Z string is the
 * diagonal sum over |psi_x|^2 with signs; a string with X or Y factors is
 * Re <psi|P psi> with P applied to a copy (tmp, 2^n entries). */
static void expvals(const circ_t *c, const cplx *psi, double *out, cplx *tmp, int par) {
  const int64_t dim = (int64_t)1 << c->n;
  for (int m = 0; m < c->n_obs; ++m) {
    double acc = 0.0;
    if (xmask_of(c, m)) {
      memcpy(tmp, psi, sizeof(cplx) * dim);
      apply_pauli(tmp, c->n, xmask_of(c, m), c->masks[m], par);
#pragma omp parallel for if (par) reduction(+ : acc) schedule(static)
      for (int64_t x = 0; x < dim; ++x) acc += creal(conj(psi[x]) * tmp[x]);
    } else {
#pragma omp parallel for if (par) reduction(+ : acc) schedule(static)
      for (int64_t x = 0; x < dim; ++x) {
        double p = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
        acc += zsign(x, c->masks[m]) * p;
      }
    }
    out[m] = acc;
  }
}

/* 2 Re <a|b> */
static double two_re_inner(const cplx *a, const cplx *b, int64_t dim, int par) {
  double acc = 0.0;
#pragma omp parallel for if (par) reduction(+ : acc) schedule(static)
  for (int64_t x = 0; x < dim; ++x) acc += creal(conj(a[x]) * b[x]);
  return 2.0 * acc;
}

/*
 * Reverse sweep for one sample with n_bra bras (Jones and Gacon, Algorithm 1,
 * extended to several bras).  On entry phi holds U|0> and lam[j] the j-th bra
 * (already multiplied by its observable).  For k = N..1:
 *   phi <- G_k^dag phi;
 *   if G_k is parameterised: mu = (dG_k/dt) phi, g[j][k] = 2 Re<lam_j|mu>;
 *   lam_j <- G_k^dag lam_j.
 * g_occ is [n_bra][n_gates]; entries of unparameterised gates are set to 0.
 */
static void reverse_sweep(const circ_t *c, const double *x_b, const double *w,
                          cplx *phi, cplx **lam, int n_bra, cplx *mu,
                          double *g_occ, int par) {
  const int64_t dim = (int64_t)1 << c->n;
  for (int k = c->n_gates - 1; k >= 0; --k) {
    const int32_t *g = c->gates + 5 * k;
    apply_gate(phi, c->n, g, x_b, w, 1, par);
    if (is_param(g[0])) {
      cplx d[2][2];
      memcpy(mu, phi, sizeof(cplx) * dim);
      if (is_rot(g[0])) {
        rot_deriv(g[0], angle_of(g, x_b, w), d);
        apply_1q(mu, c->n, g[1], d, par);
      } else {
        /* d/dt of |0><0| (x) I + |1><1| (x) R(t) on (control, target) is
         * |1><1| (x) dR/dt: zero where the control bit is 0 */
        const int64_t cb = (int64_t)1 << g[1];
        rot_deriv(g[0] - O_CRX, angle_of(g, x_b, w), d);
        for (int64_t x = 0; x < dim; ++x)
          if (!(x & cb)) mu[x] = 0;
        apply_1q_ctl(mu, c->n, g[1], g[2], d, par);
      }
      for (int j = 0; j < n_bra; ++j)
        g_occ[(int64_t)j * c->n_gates + k] = two_re_inner(lam[j], mu, dim, par);
    } else {
      for (int j = 0; j < n_bra; ++j) g_occ[(int64_t)j * c->n_gates + k] = 0.0;
    }
    for (int j = 0; j < n_bra; ++j) apply_gate(lam[j], c->n, g, x_b, w, 1, par);
  }
}

/* Sample range of thread t under the batch split of Sec. II-B. */
static void split_range(int B, int T, int t, int *lo, int *hi) {
  int base = B / T, rem = B - T * base;
  *lo = t * base + (t < rem ? t : rem);
  *hi = *lo + base + (t < rem ? 1 : 0);
}

int qtm_oracle_split(int B, int T, int t, int32_t *lo_hi) {
  if (B < 0 || T < 1 || t < 0 || t >= T) return -1;
  int lo, hi;
  split_range(B, T, t, &lo, &hi);
  lo_hi[0] = lo;
  lo_hi[1] = hi;
  return 0;
}

/* Work item shared by the entry points.  mode 0: expectation values only;
 * mode 1: VJP with the combined bra; mode 2: full Jacobian with M bras. */
typedef struct {
  const circ_t *c;
  const double *x, *w, *G;
  double *out, *gw_per_sample, *gx, *g_occ, *jw, *jx;
  int mode;
} job_t;

static int run_sample(const job_t *J, int b, int par) {
  const circ_t *c = J->c;
  const int64_t dim = (int64_t)1 << c->n;
  const double *x_b = J->x + (int64_t)b * c->n_inputs;
  const int M = c->n_obs;
  cplx *phi = malloc(sizeof(cplx) * dim);
  cplx *mu = malloc(sizeof(cplx) * dim);
  if (!phi || !mu) return -2;
  evolve(c, x_b, J->w, phi, par);
  if (J->out) expvals(c, phi, J->out + (int64_t)b * M, mu, par);
  if (J->mode == 0) {
    free(phi);
    free(mu);
    return 0;
  }
  int n_bra = J->mode == 1 ? 1 : M;
  cplx **lam = malloc(sizeof(cplx *) * (n_bra > 0 ? n_bra : 1));
  double *g = calloc((size_t)(n_bra > 0 ? n_bra : 1) * (c->n_gates > 0 ? c->n_gates : 1), sizeof(double));
  int ok = lam && g;
  for (int j = 0; ok && j < n_bra; ++j) ok = (lam[j] = malloc(sizeof(cplx) * dim)) != NULL;
  if (!ok) return -2; /* test infrastructure: leak on OOM is acceptable */
  /* bras: lambda = (sum_m G_m O_m) phi  or  lambda_m = O_m phi; the Z
   * strings as one diagonal, every string with X or Y factors added as
   * G_m (P_m phi) (P_m applied to a copy of phi in mu) */
  for (int j = 0; j < n_bra; ++j) {
#pragma omp parallel for if (par) schedule(static)
    for (int64_t x = 0; x < dim; ++x) {
      double dsum = 0.0;
      if (J->mode == 1) {
        for (int m = 0; m < M; ++m)
          if (!xmask_of(c, m)) dsum += J->G[(int64_t)b * M + m] * zsign(x, c->masks[m]);
      } else if (!xmask_of(c, j)) {
        dsum = zsign(x, c->masks[j]);
      }
      lam[j][x] = dsum * phi[x];
    }
    for (int m = 0; m < M; ++m) {
      if (!xmask_of(c, m) || (J->mode == 2 && m != j)) continue;
      const double gm = J->mode == 1 ? J->G[(int64_t)b * M + m] : 1.0;
      memcpy(mu, phi, sizeof(cplx) * dim);
      apply_pauli(mu, c->n, xmask_of(c, m), c->masks[m], par);
#pragma omp parallel for if (par) schedule(static)
      for (int64_t x = 0; x < dim; ++x) lam[j][x] += gm * mu[x];
    }
  }
  reverse_sweep(c, x_b, J->w, phi, lam, n_bra, mu, g, par);
  /* scatter per-occurrence derivatives into parameter slots (Eq. (5)-(6)) */
  for (int j = 0; j < n_bra; ++j) {
    for (int k = 0; k < c->n_gates; ++k) {
      const int32_t *gk = c->gates + 5 * k;
      if (!is_param(gk[0])) continue;
      double v = g[(int64_t)j * c->n_gates + k];
      /* d angle / d parameter: 1, or for a scaled input the other factor */
      double *wrow = J->mode == 1 ? J->gw_per_sample + (int64_t)b * c->n_weights
                                  : J->jw + ((int64_t)b * M + j) * c->n_weights;
      double *xrow = J->mode == 1 ? (J->gx ? J->gx + (int64_t)b * c->n_inputs : NULL)
                                  : J->jx + ((int64_t)b * M + j) * c->n_inputs;
      if (J->mode == 1 && J->g_occ) J->g_occ[(int64_t)b * c->n_gates + k] = v;
      if (gk[3] == O_SRC_WEIGHT) {
        wrow[gk[4]] += v;
      } else if (gk[3] == O_SRC_INPUT) {
        if (xrow) xrow[gk[4]] += v;
      } else {
        wrow[gk[2]] += v * x_b[gk[4]];
        if (xrow) xrow[gk[4]] += v * J->w[gk[2]];
      }
    }
  }
  for (int j = 0; j < n_bra; ++j) free(lam[j]);
  free(lam);
  free(g);
  free(mu);
  free(phi);
  return 0;
}

/* par_mode 0: samples split over `threads` threads (Sec. II-B rule);
 * par_mode 1: samples one after another, each gate loop over `threads`. */
static int run_batch(const job_t *J, int B, int threads, int par_mode) {
  if (threads < 1) threads = 1;
  int err = 0;
  if (par_mode == 1) {
    omp_set_num_threads(threads);
    for (int b = 0; b < B && !err; ++b) err = run_sample(J, b, 1);
    return err;
  }
#pragma omp parallel num_threads(threads) reduction(| : err)
  {
    int T = omp_get_num_threads(), t = omp_get_thread_num(), lo, hi;
    split_range(B, T, t, &lo, &hi);
    for (int b = lo; b < hi; ++b) err |= run_sample(J, b, 0) ? 1 : 0;
  }
  return err ? -2 : 0;
}

int qtm_oracle_forward(int n, const int32_t *gates, int n_gates, int n_inputs,
                       int n_weights, const uint64_t *masks, const uint64_t *xmasks, int n_obs, int B,
                       const double *x, const double *w, double *out,
                       int threads, int par_mode) {
  circ_t c = {n, gates, n_gates, n_inputs, n_weights, masks, n_obs, xmasks};
  if (check_circuit(&c) || B < 0 || !out) return -1;
  job_t J = {&c, x, w, NULL, out, NULL, NULL, NULL, NULL, NULL, 0};
  return run_batch(&J, B, threads, par_mode);
}

/* VJP: grad_w[j] = sum_b sum_m G[b][m] d<O_m>_b/dw_j;
 *      grad_x[b][i] = sum_m G[b][m] d<O_m>_b/dx_{b,i}.
 * out (expectation values), grad_x and g_occ ([B][n_gates], per gate
 * occurrence) may be NULL. */
int qtm_oracle_vjp(int n, const int32_t *gates, int n_gates, int n_inputs,
                   int n_weights, const uint64_t *masks, const uint64_t *xmasks, int n_obs, int B,
                   const double *x, const double *w, const double *G,
                   double *out, double *grad_w, double *grad_x, double *g_occ,
                   int threads, int par_mode) {
  circ_t c = {n, gates, n_gates, n_inputs, n_weights, masks, n_obs, xmasks};
  if (check_circuit(&c) || B < 0 || !grad_w || !G) return -1;
  double *gws = calloc((size_t)(B > 0 ? B : 1) * (n_weights > 0 ? n_weights : 1), sizeof(double));
  if (!gws) return -2;
  if (grad_x) memset(grad_x, 0, sizeof(double) * (size_t)B * n_inputs);
  if (g_occ) memset(g_occ, 0, sizeof(double) * (size_t)B * n_gates);
  job_t J = {&c, x, w, G, out, gws, grad_x, g_occ, NULL, NULL, 1};
  int err = run_batch(&J, B, threads, par_mode);
  /* batch sum of the weight gradient, samples in order */
  for (int j = 0; j < n_weights; ++j) {
    double acc = 0.0;
    for (int b = 0; b < B; ++b) acc += gws[(int64_t)b * n_weights + j];
    grad_w[j] = acc;
  }
  free(gws);
  return err;
}

/* Full Jacobian (B, M, |Theta|) of Sec. II-B: jw [B][M][n_weights],
 * jx [B][M][n_inputs]; out may be NULL. */
int qtm_oracle_jacobian(int n, const int32_t *gates, int n_gates, int n_inputs,
                        int n_weights, const uint64_t *masks, const uint64_t *xmasks, int n_obs, int B,
                        const double *x, const double *w, double *out,
                        double *jw, double *jx, int threads, int par_mode) {
  circ_t c = {n, gates, n_gates, n_inputs, n_weights, masks, n_obs, xmasks};
  if (check_circuit(&c) || B < 0 || !jw || !jx) return -1;
  memset(jw, 0, sizeof(double) * (size_t)B * n_obs * n_weights);
  memset(jx, 0, sizeof(double) * (size_t)B * n_obs * n_inputs);
  job_t J = {&c, x, w, NULL, out, NULL, NULL, NULL, jw, jx, 2};
  return run_batch(&J, B, threads, par_mode);
}

/* Final state U|0> of one sample, as interleaved (re, im) doubles. */
int qtm_oracle_state(int n, const int32_t *gates, int n_gates, int n_inputs,
                     int n_weights, const double *x_b, const double *w,
                     double *state) {
  circ_t c = {n, gates, n_gates, n_inputs, n_weights, NULL, 0, NULL};
  if (check_circuit(&c) || !state) return -1;
  const int64_t dim = (int64_t)1 << n;
  cplx *psi = malloc(sizeof(cplx) * dim);
  if (!psi) return -2;
  evolve(&c, x_b, w, psi, 0);
  for (int64_t x = 0; x < dim; ++x) {
    state[2 * x] = creal(psi[x]);
    state[2 * x + 1] = cimag(psi[x]);
  }
  free(psi);
  return 0;
}

/* Uncompute check: evolve, then un-apply every gate in reverse; returns
 * |psi[0]| of the result through *amp0 (1 up to rounding). */
int qtm_oracle_uncompute(int n, const int32_t *gates, int n_gates, int n_inputs,
                         int n_weights, const double *x_b, const double *w,
                         double *amp0) {
  circ_t c = {n, gates, n_gates, n_inputs, n_weights, NULL, 0, NULL};
  if (check_circuit(&c) || !amp0) return -1;
  const int64_t dim = (int64_t)1 << n;
  cplx *psi = malloc(sizeof(cplx) * dim);
  if (!psi) return -2;
  evolve(&c, x_b, w, psi, 0);
  for (int k = n_gates - 1; k >= 0; --k) apply_gate(psi, n, gates + 5 * k, x_b, w, 1, 0);
  *amp0 = cabs(psi[0]);
  free(psi);
  return 0;
}
