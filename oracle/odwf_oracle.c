/*
 * FP64 CPU oracle for the optimal domain-wall fermion operator and its
 * even-odd preconditioned conjugate-gradient solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library: gamma matrices, projectors, the
 * fifth-dimension matrices and every loop are written out here from the
 * definitions, in double precision, with no blocking or fusion.
 *
 * Paper: T.-W. Chiu, "Simulation of dynamical (u,d,s,c) domain-wall/overlap
 * quarks at the physical point", LATTICE2018 (arXiv:1811.08095).
 *   - §2: the operator D_odwf(m_q) is the optimal domain-wall operator with
 *     c = 1, d = 0 (so H = H_w, the Hermitian Wilson operator), m0 = 1.3,
 *     N_s = 16, R5-symmetric weights omega_s, m_PV = 2 m0.  The paper defers the
 *     explicit matrix to its reference [Chiu:2013aaa, Eq. (2)]; the form used
 *     here is the c = 1, d = 0 case of that operator:
 *         D = omega D_w (1 + L) + (1 - L),
 *         L = P_- L_- + P_+ L_+,  P_pm = (1 pm gamma5)/2,
 *         (L_+ psi)_s = psi_{s-1} (s > 1),   (L_+ psi)_1   = -mu psi_{N_s},
 *         (L_- psi)_s = psi_{s+1} (s < N_s), (L_- psi)_{N_s} = -mu psi_1,
 *     with mu = m_q / m_PV = m_q / (2 m0), so that D(m_PV) is the mu = 1 operator
 *     of the Pauli-Villars factors of Eq. (1)-(2).
 *   - D_w is the 4D Wilson-Dirac operator with negative mass -m0 and r = 1:
 *         (D_w psi)(x) = (4 - m0) psi(x)
 *           - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                        + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ].
 *     Every hop that crosses the t boundary is multiplied by bc_t (+1 or -1).
 *   - Even-odd preconditioning is not in the paper.  With W = D_w - (4 - m0)
 *     and A = (4 - m0) + omega^{-1} (1 - L)(1 + L)^{-1} (site-local),
 *     D x = b  <=>  (A + W) y = omega^{-1} b,  x = (1 + L)^{-1} y,
 *     and the even-site Schur complement in unit-diagonal form is
 *         S_e = 1 - A^{-1} W_eo A^{-1} W_oe,
 *         phi_e = A^{-1} (b'_e - W_eo A^{-1} b'_o),
 *         y_o   = A^{-1} (b'_o - W_oe y_e).
 *   - §2 (conjugate gradient): the solve is textbook Hestenes-Stiefel CG on
 *     the Hermitian positive-definite normal operator S_e^dag S_e.
 *
 * Mutation testing: building with -DORACLE_PLANT=k (k = 1..14) plants one
 * deliberate, plausible mistake (see PLANT below) so that the tests can show
 * that their pins reject it; the normal build never defines it.
 *
 * Conventions: gamma matrices in the chiral basis
 *     gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),
 *     gamma_4 = [[0, 1], [1, 0]],   gamma5 = gamma1 gamma2 gamma3 gamma4.
 * Spinor fields (one right-hand side): complex128 [s][t][z][y][x][spin 4][color 3].
 * Gauge field: complex128 [t][z][y][x][mu = x,y,z,t][3][3], U_mu(x) links x to x+mu.
 * Parity of a site is (x + y + z + t) mod 2; 0 = even.
 */
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif
#define PLANT(k) (ORACLE_PLANT == (k))

enum {
  OR_OP_HOP_EO = 0,
  OR_OP_HOP_OE = 1,
  OR_OP_M5INV = 2,
  OR_OP_D = 3,
  OR_OP_DDAG = 4,
  OR_OP_DDAGD = 5,
  OR_OP_SCHUR = 6,
  OR_OP_SCHUR_DAG = 7,
  OR_OP_SCHUR_NORMAL = 8,
};

enum { OR_SOLVE_EO_NORMAL = 0, OR_SOLVE_FULL = 1 };

/* ------------------------------------------------------------------------ */
/* gamma matrices, written from the chiral-basis definition                  */
/* ------------------------------------------------------------------------ */

static cplx G[4][4][4]; /* gamma_mu, mu = 0..3 for x,y,z,t */
static cplx G5[4][4];
static int gamma_ready = 0;

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx c[4][4]) {
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) {
      cplx s = 0;
      for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
      c[i][j] = s;
    }
}

static void init_gamma(void) {
  if (gamma_ready) return;
  /* Pauli matrices */
  cplx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  memset(G, 0, sizeof(G));
  for (int k = 0; k < 3; k++)
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) {
        G[k][a][2 + b] = -I * sig[k][a][b]; /* upper-right block: -i sigma_k */
        G[k][2 + a][b] = I * sig[k][a][b];  /* lower-left block:  +i sigma_k */
      }
  for (int a = 0; a < 2; a++) {
    G[3][a][2 + a] = 1;
    G[3][2 + a][a] = 1;
  }
  cplx t1[4][4], t2[4][4];
  mat4_mul(G[0], G[1], t1);
  mat4_mul(t1, G[2], t2);
  mat4_mul(t2, G[3], G5);
  gamma_ready = 1;
}

/* ------------------------------------------------------------------------ */
/* lattice geometry                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int L[4];
  long V;
  int bc_t;
} geom_t;

static geom_t make_geom(const int dims[4], int bc_t) {
  geom_t g;
  for (int m = 0; m < 4; m++) g.L[m] = dims[m];
  g.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  g.bc_t = bc_t;
  return g;
}

static void site_coords(const geom_t* g, long i, int c[4]) {
  for (int m = 0; m < 4; m++) {
    c[m] = (int)(i % g->L[m]);
    i /= g->L[m];
  }
}

static long site_index(const geom_t* g, const int c[4]) {
  return ((long)(c[3] * g->L[2] + c[2]) * g->L[1] + c[1]) * g->L[0] + c[0];
}

static int site_parity(const geom_t* g, long i) {
  int c[4];
  site_coords(g, i, c);
  return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* neighbour of site i in direction mu, step +1 or -1; *sign receives the
 * boundary factor (bc_t when the hop wraps around in t, else +1). */
static long neighbour(const geom_t* g, long i, int mu, int step, double* sign) {
  int c[4];
  site_coords(g, i, c);
  int v = c[mu] + (PLANT(9) && mu == 2 ? -step : step);
  *sign = 1.0;
  if (v >= g->L[mu]) {
    v -= g->L[mu];
    if (mu == 3) *sign = g->bc_t;
  } else if (v < 0) {
    v += g->L[mu];
    if (mu == 3) *sign = g->bc_t;
  }
  c[mu] = v;
  return site_index(g, c);
}

/* ------------------------------------------------------------------------ */
/* 4D Wilson hopping term                                                   */
/* ------------------------------------------------------------------------ */

/* (W psi)(x) = -1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                          + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * dag != 0 gives the adjoint W^dag, obtained by taking the Hermitian
 * conjugate of each matrix element: the projectors swap,
 * (W^dag psi)(x) = -1/2 sum_mu [ (1 + gamma_mu) U_mu(x) psi(x+mu)
 *                              + (1 - gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].
 * in/out: one 4D spinor field [V][4][3].  Sites where out_mask says 0 are
 * left at zero; input sites where in_mask says 0 are treated as zero. */
static void wilson_hop_4d(const geom_t* g, const cplx* U, int dag, const cplx* in,
                          cplx* out, int out_par, int in_par) {
  init_gamma();
  double fwd_sign = dag ? +1.0 : -1.0; /* sign of gamma_mu on the forward hop */
  if (PLANT(1)) fwd_sign = -fwd_sign;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < g->V; x++) {
    cplx acc[4][3];
    memset(acc, 0, sizeof(acc));
    int px = site_parity(g, x);
    if (out_par >= 0 && px != out_par) {
      memset(out + x * 12, 0, sizeof(cplx) * 12);
      continue;
    }
    for (int mu = 0; mu < 4; mu++) {
      for (int dir = 0; dir < 2; dir++) {
        double bsign;
        long y = neighbour(g, x, mu, dir == 0 ? +1 : -1, &bsign);
        if (in_par >= 0 && site_parity(g, y) != in_par) continue;
        /* link: forward U_mu(x); backward U_mu(x - mu)^dag */
        cplx link[3][3];
        if (dir == 0) {
          const cplx* u = U + (x * 4 + mu) * 9;
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) link[a][b] = u[a * 3 + b];
        } else {
          const cplx* u = U + (y * 4 + mu) * 9;
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) link[a][b] = PLANT(2) ? u[a * 3 + b] : conj(u[b * 3 + a]);
        }
        /* projector (1 + s gamma_mu): forward s = fwd_sign, backward -fwd_sign */
        double s = dir == 0 ? fwd_sign : -fwd_sign;
        cplx proj[4][4];
        for (int a = 0; a < 4; a++)
          for (int b = 0; b < 4; b++) proj[a][b] = (a == b ? 1.0 : 0.0) + s * G[mu][a][b];
        const cplx* p = in + y * 12;
        /* color rotation, then spin projection */
        cplx up[4][3];
        for (int sp = 0; sp < 4; sp++)
          for (int a = 0; a < 3; a++) {
            cplx v = 0;
            for (int b = 0; b < 3; b++) v += link[a][b] * p[sp * 3 + b];
            up[sp][a] = v;
          }
        for (int sp = 0; sp < 4; sp++)
          for (int a = 0; a < 3; a++) {
            cplx v = 0;
            for (int t = 0; t < 4; t++) v += proj[sp][t] * up[t][a];
            acc[sp][a] += (PLANT(8) ? -1.0 : -0.5) * (PLANT(3) ? 1.0 : bsign) * v;
          }
      }
    }
    for (int sp = 0; sp < 4; sp++)
      for (int a = 0; a < 3; a++) out[x * 12 + sp * 3 + a] = acc[sp][a];
  }
}

/* ------------------------------------------------------------------------ */
/* dense linear algebra on small matrices (fifth dimension x spin)          */
/* ------------------------------------------------------------------------ */

/* Gauss-Jordan inverse with partial pivoting; n x n complex, row major. */
static int cinv(int n, const cplx* a, cplx* ainv) {
  cplx* m = malloc(sizeof(cplx) * n * 2 * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < 2 * n; j++) m[i * 2 * n + j] = j < n ? a[i * n + j] : (j - n == i ? 1 : 0);
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (cabs(m[r * 2 * n + c]) > cabs(m[piv * 2 * n + c])) piv = r;
    if (cabs(m[piv * 2 * n + c]) == 0) {
      free(m);
      return -1;
    }
    if (piv != c)
      for (int j = 0; j < 2 * n; j++) {
        cplx t = m[c * 2 * n + j];
        m[c * 2 * n + j] = m[piv * 2 * n + j];
        m[piv * 2 * n + j] = t;
      }
    cplx d = m[c * 2 * n + c];
    for (int j = 0; j < 2 * n; j++) m[c * 2 * n + j] /= d;
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      cplx f = m[r * 2 * n + c];
      if (f == 0) continue;
      for (int j = 0; j < 2 * n; j++) m[r * 2 * n + j] -= f * m[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) ainv[i * n + j] = m[i * 2 * n + n + j];
  free(m);
  return 0;
}

static void cmatmul(int n, const cplx* a, const cplx* b, cplx* c) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      cplx s = 0;
      for (int k = 0; k < n; k++) s += a[i * n + k] * b[k * n + j];
      c[i * n + j] = s;
    }
}

static void cadjoint(int n, const cplx* a, cplx* b) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) b[i * n + j] = conj(a[j * n + i]);
}

/* The operators on the (s, spin) space of dimension n = 4 Ns, index s*4+spin.
 * which: 0 = L, 1 = (1 + L)^{-1}, 2 = A, 3 = A^{-1}, 4 = omega, 5 = omega^{-1}. */
static int m5_matrix(int Ns, double m0, const double* omega, double mu, int which, cplx* out) {
  init_gamma();
  int n = 4 * Ns;
  cplx Pp[4][4], Pm[4][4];
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) {
      Pp[a][b] = 0.5 * ((a == b ? 1.0 : 0.0) + G5[a][b]);
      Pm[a][b] = 0.5 * ((a == b ? 1.0 : 0.0) - G5[a][b]);
    }
  double* Lp = calloc((size_t)Ns * Ns, sizeof(double));
  double* Lm = calloc((size_t)Ns * Ns, sizeof(double));
  for (int s = 1; s < Ns; s++) Lp[s * Ns + s - 1] = 1.0;
  Lp[0 * Ns + Ns - 1] = PLANT(4) ? mu : -mu;
  for (int s = 0; s < Ns - 1; s++) Lm[s * Ns + s + 1] = 1.0;
  Lm[(Ns - 1) * Ns + 0] = PLANT(4) ? mu : -mu;
  cplx* L = calloc((size_t)n * n, sizeof(cplx));
  for (int s = 0; s < Ns; s++)
    for (int t = 0; t < Ns; t++)
      for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
          L[(s * 4 + a) * n + t * 4 + b] = PLANT(5) ? Lm[s * Ns + t] * Pm[a][b] + Lm[s * Ns + t] * Pp[a][b]
                                                    : Lm[s * Ns + t] * Pm[a][b] + Lp[s * Ns + t] * Pp[a][b];
  int rc = 0;
  cplx* one_plus = calloc((size_t)n * n, sizeof(cplx));
  cplx* one_minus = calloc((size_t)n * n, sizeof(cplx));
  cplx* inv_one_plus = calloc((size_t)n * n, sizeof(cplx));
  cplx* tmp = calloc((size_t)n * n, sizeof(cplx));
  cplx* A = calloc((size_t)n * n, sizeof(cplx));
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      one_plus[i * n + j] = (i == j ? 1.0 : 0.0) + L[i * n + j];
      one_minus[i * n + j] = (i == j ? 1.0 : 0.0) - L[i * n + j];
    }
  rc |= cinv(n, one_plus, inv_one_plus);
  cmatmul(n, one_minus, inv_one_plus, tmp);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++)
      A[i * n + j] = (i == j ? (4.0 - m0) : 0.0) + tmp[i * n + j] / omega[i / 4];
  switch (which) {
    case 0: memcpy(out, L, sizeof(cplx) * n * n); break;
    case 1: memcpy(out, inv_one_plus, sizeof(cplx) * n * n); break;
    case 2: memcpy(out, A, sizeof(cplx) * n * n); break;
    case 3: rc |= cinv(n, A, out); break;
    case 4:
    case 5:
      memset(out, 0, sizeof(cplx) * n * n);
      for (int i = 0; i < n; i++) out[i * n + i] = which == 4 ? omega[i / 4] : 1.0 / omega[i / 4];
      break;
    default: rc = -1;
  }
  free(Lp); free(Lm); free(L); free(one_plus); free(one_minus);
  free(inv_one_plus); free(tmp); free(A);
  return rc;
}

/* apply an (s, spin) matrix M (n = 4 Ns) at every site and color of a 5D field;
 * sites of the wrong parity (par >= 0) are set to zero. */
static void apply_m5(const geom_t* g, int Ns, const cplx* M, const cplx* in, cplx* out, int par) {
  int n = 4 * Ns;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < g->V; x++) {
    int keep = par < 0 || site_parity(g, x) == par;
    for (int s = 0; s < Ns; s++)
      for (int a = 0; a < 4; a++)
        for (int c = 0; c < 3; c++) {
          cplx v = 0;
          if (keep)
            for (int t = 0; t < Ns; t++)
              for (int b = 0; b < 4; b++)
                v += M[(s * 4 + a) * n + t * 4 + b] * in[((long)t * g->V + x) * 12 + b * 3 + c];
          out[((long)s * g->V + x) * 12 + a * 3 + c] = v;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* vector helpers on 5D fields                                              */
/* ------------------------------------------------------------------------ */

static cplx vdot(long n, const cplx* a, const cplx* b) {
  double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
  for (long i = 0; i < n; i++) {
    cplx p = conj(a[i]) * b[i];
    re += creal(p);
    im += cimag(p);
  }
  return re + I * im;
}

static double vnorm2(long n, const cplx* a) { return creal(vdot(n, a, a)); }

/* zero the sites of parity par in a 5D field */
static void mask_parity(const geom_t* g, int Ns, cplx* v, int par) {
#pragma omp parallel for schedule(static)
  for (long x = 0; x < g->V; x++)
    if (site_parity(g, x) == par)
      for (int s = 0; s < Ns; s++) memset(v + ((long)s * g->V + x) * 12, 0, sizeof(cplx) * 12);
}

/* ------------------------------------------------------------------------ */
/* the operator context                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  geom_t g;
  const cplx* U;
  int Ns;
  double m0;
  const double* omega;
  double mu;
  long n5; /* complex entries of a 5D field */
  cplx *L, *A, *Ainv, *AinvDag, *onePlusLinv;
} ctx_t;

static int ctx_init(ctx_t* c, const int dims[4], int bc_t, const cplx* U, int Ns, double m0,
                    const double* omega, double mu) {
  c->g = make_geom(dims, bc_t);
  c->U = U;
  c->Ns = Ns;
  c->m0 = m0;
  c->omega = omega;
  c->mu = mu;
  c->n5 = (long)Ns * c->g.V * 12;
  int n = 4 * Ns;
  c->L = malloc(sizeof(cplx) * n * n);
  c->A = malloc(sizeof(cplx) * n * n);
  c->Ainv = malloc(sizeof(cplx) * n * n);
  c->AinvDag = malloc(sizeof(cplx) * n * n);
  c->onePlusLinv = malloc(sizeof(cplx) * n * n);
  int rc = m5_matrix(Ns, m0, omega, mu, 0, c->L);
  rc |= m5_matrix(Ns, m0, omega, mu, 2, c->A);
  rc |= m5_matrix(Ns, m0, omega, mu, 3, c->Ainv);
  rc |= m5_matrix(Ns, m0, omega, mu, 1, c->onePlusLinv);
  cadjoint(n, c->Ainv, c->AinvDag);
  return rc;
}

static void ctx_free(ctx_t* c) {
  free(c->L); free(c->A); free(c->Ainv); free(c->AinvDag); free(c->onePlusLinv);
}

/* W on a 5D field, s by s; out_par / in_par as in wilson_hop_4d */
static void hop5(const ctx_t* c, int dag, const cplx* in, cplx* out, int out_par, int in_par) {
  for (int s = 0; s < c->Ns; s++)
    wilson_hop_4d(&c->g, c->U, dag, in + (long)s * c->g.V * 12, out + (long)s * c->g.V * 12,
                  out_par, in_par);
}

/* D psi = omega D_w (1 + L) psi + (1 - L) psi */
static void op_D(const ctx_t* c, const cplx* in, cplx* out) {
  long n = c->n5;
  cplx* Lpsi = malloc(sizeof(cplx) * n);
  cplx* y = malloc(sizeof(cplx) * n);
  cplx* dw = malloc(sizeof(cplx) * n);
  apply_m5(&c->g, c->Ns, c->L, in, Lpsi, -1);
  for (long i = 0; i < n; i++) y[i] = in[i] + Lpsi[i];
  hop5(c, 0, y, dw, -1, -1);
  long vs = c->g.V * 12;
  for (long i = 0; i < n; i++) {
    double w = c->omega[i / vs];
    out[i] = w * (dw[i] + ((PLANT(6) ? 5.0 : 4.0) - c->m0) * y[i]) + in[i] - Lpsi[i];
  }
  free(Lpsi); free(y); free(dw);
}

/* D^dag psi = (1 + L)^dag D_w^dag (omega psi) + (1 - L)^dag psi */
static void op_Ddag(const ctx_t* c, const cplx* in, cplx* out) {
  long n = c->n5;
  int m = 4 * c->Ns;
  long vs = c->g.V * 12;
  cplx* Ldag = malloc(sizeof(cplx) * m * m);
  cadjoint(m, c->L, Ldag);
  cplx* w = calloc((size_t)n, sizeof(cplx)); /* every entry is set below */
  cplx* dw = malloc(sizeof(cplx) * n);
  cplx* t1 = malloc(sizeof(cplx) * n);
  cplx* t2 = malloc(sizeof(cplx) * n);
  for (long i = 0; i < n; i++) w[i] = c->omega[i / vs] * in[i];
  hop5(c, 1, w, dw, -1, -1);
  for (long i = 0; i < n; i++) dw[i] += (4.0 - c->m0) * w[i];
  apply_m5(&c->g, c->Ns, Ldag, dw, t1, -1);
  apply_m5(&c->g, c->Ns, Ldag, in, t2, -1);
  for (long i = 0; i < n; i++) out[i] = dw[i] + t1[i] + in[i] - t2[i];
  free(Ldag); free(w); free(dw); free(t1); free(t2);
}

/* S_e psi_e = psi_e - A^{-1} W_eo A^{-1} W_oe psi_e ; odd sites of out are 0 */
static void op_schur(const ctx_t* c, const cplx* in, cplx* out) {
  long n = c->n5;
  cplx* t1 = malloc(sizeof(cplx) * n);
  cplx* t2 = malloc(sizeof(cplx) * n);
  hop5(c, 0, in, t1, 1, 0);                       /* W_oe psi_e        (odd)  */
  apply_m5(&c->g, c->Ns, c->Ainv, t1, t2, 1);     /* A^{-1} ...        (odd)  */
  hop5(c, 0, t2, t1, 0, 1);                       /* W_eo ...          (even) */
  apply_m5(&c->g, c->Ns, c->Ainv, t1, t2, 0);     /* A^{-1} ...        (even) */
  cplx* e = malloc(sizeof(cplx) * n);
  memcpy(e, in, sizeof(cplx) * n);
  mask_parity(&c->g, c->Ns, e, 1);
  for (long i = 0; i < n; i++) out[i] = PLANT(7) ? e[i] + t2[i] : e[i] - t2[i];
  free(t1); free(t2); free(e);
}

/* S_e^dag psi_e = psi_e - (W_oe)^dag (A^{-1})^dag (W_eo)^dag (A^{-1})^dag psi_e.
 * (W_eo)^dag maps even to odd and is the odd-even block of W^dag. */
static void op_schur_dag(const ctx_t* c, const cplx* in, cplx* out) {
  long n = c->n5;
  cplx* t1 = malloc(sizeof(cplx) * n);
  cplx* t2 = malloc(sizeof(cplx) * n);
  apply_m5(&c->g, c->Ns, c->AinvDag, in, t1, 0);  /* (A^{-1})^dag psi_e  (even) */
  hop5(c, 1, t1, t2, 1, 0);                       /* (W_eo)^dag ...      (odd)  */
  apply_m5(&c->g, c->Ns, c->AinvDag, t2, t1, 1);  /* (A^{-1})^dag ...    (odd)  */
  hop5(c, 1, t1, t2, 0, 1);                       /* (W_oe)^dag ...      (even) */
  cplx* e = malloc(sizeof(cplx) * n);
  memcpy(e, in, sizeof(cplx) * n);
  mask_parity(&c->g, c->Ns, e, 1);
  for (long i = 0; i < n; i++) out[i] = e[i] - t2[i];
  free(t1); free(t2); free(e);
}

static void op_schur_normal(const ctx_t* c, const cplx* in, cplx* out) {
  cplx* t = malloc(sizeof(cplx) * c->n5);
  op_schur(c, in, t);
  op_schur_dag(c, t, out);
  free(t);
}

static int apply_op(const ctx_t* c, int op, const cplx* in, cplx* out) {
  long n = c->n5;
  switch (op) {
    case OR_OP_HOP_EO: hop5(c, 0, in, out, PLANT(10) ? 1 : 0, PLANT(10) ? 0 : 1); return 0;
    case OR_OP_HOP_OE: hop5(c, 0, in, out, PLANT(10) ? 0 : 1, PLANT(10) ? 1 : 0); return 0;
    case OR_OP_M5INV:
      if (PLANT(12)) { /* the transposed matrix */
        int m = 4 * c->Ns;
        cplx* T = malloc(sizeof(cplx) * m * m);
        for (int i = 0; i < m; i++)
          for (int j = 0; j < m; j++) T[i * m + j] = c->Ainv[j * m + i];
        apply_m5(&c->g, c->Ns, T, in, out, -1);
        free(T);
        return 0;
      }
      apply_m5(&c->g, c->Ns, c->Ainv, in, out, -1);
      return 0;
    case OR_OP_D: op_D(c, in, out); return 0;
    case OR_OP_DDAG: op_Ddag(c, in, out); return 0;
    case OR_OP_DDAGD: {
      cplx* t = malloc(sizeof(cplx) * n);
      op_D(c, in, t);
      op_Ddag(c, t, out);
      free(t);
      return 0;
    }
    case OR_OP_SCHUR: op_schur(c, in, out); return 0;
    case OR_OP_SCHUR_DAG: op_schur_dag(c, in, out); return 0;
    case OR_OP_SCHUR_NORMAL: op_schur_normal(c, in, out); return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                    */
/* ------------------------------------------------------------------------ */

/* number of threads the oracle's parallel loops use */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* gamma matrices as the oracle builds them: out[5][4][4] (gamma_1..4, gamma5) */
void oracle_gammas(cplx* out) {
  init_gamma();
  memcpy(out, G, sizeof(G));
  memcpy(out + 64, G5, sizeof(G5));
}

/* 4D Wilson-Dirac operator on one 4D field: out = D_w in (dag = 0) or
 * D_w^dag in (dag = 1). */
int oracle_dw(const int dims[4], int bc_t, const cplx* U, double m0, int dag, const cplx* in,
              cplx* out) {
  geom_t g = make_geom(dims, bc_t);
  wilson_hop_4d(&g, U, dag, in, out, -1, -1);
  for (long i = 0; i < g.V * 12; i++) out[i] += (4.0 - m0) * in[i];
  return 0;
}

/* (s, spin) matrices, n = 4 Ns, row major: see m5_matrix */
int oracle_m5_matrix(int Ns, double m0, const double* omega, double mu, int which, cplx* out) {
  return m5_matrix(Ns, m0, omega, mu, which, out);
}

/* Fermion force of the bilinear S = Re <chi, W psi> (W the hopping term of
 * D_w, applied slice by slice and summed over s): for every link U_mu(x),
 *   M = -1/2 b sum_s ( A + B^dag ),
 *   A[b][a] = sum_spin [(1 - gamma_mu) psi(x + mu, s)]_{spin, b} conj(chi(x, s)_{spin, a}),
 *   B[b][a] = sum_spin [(1 + gamma_mu) psi(x, s)]_{spin, b} conj(chi(x + mu, s)_{spin, a}),
 * with b the boundary factor of the link (bc_t when x + mu wraps in t), so
 * that S contains Re tr(U_mu(x) M) and nothing else depends on U_mu(x); then
 *   F_mu(x) = TA(U_mu(x) M),   TA(X) = (X - X^dag)/2 - tr(X - X^dag)/6,
 * which satisfies dS/d eps = i tr(T F_mu(x)) for U_mu(x) -> exp(i eps T) U_mu(x),
 * T Hermitian and traceless.  chi, psi: [s][t][z][y][x][4][3]; F: [t][z][y][x][mu][3][3]. */
int oracle_force(const int dims[4], int bc_t, const cplx* U, int Ns, const cplx* chi, const cplx* psi,
                 cplx* F) {
  geom_t g = make_geom(dims, bc_t);
  init_gamma();
#pragma omp parallel for schedule(static)
  for (long x = 0; x < g.V; x++) {
    for (int mu = 0; mu < 4; mu++) {
      double bs;
      long y = neighbour(&g, x, mu, +1, &bs);
      cplx A[3][3], B[3][3];
      memset(A, 0, sizeof(A));
      memset(B, 0, sizeof(B));
      for (int s = 0; s < Ns; s++) {
        const cplx* py = psi + ((long)s * g.V + y) * 12;
        const cplx* px = psi + ((long)s * g.V + x) * 12;
        const cplx* cx = chi + ((long)s * g.V + x) * 12;
        const cplx* cy = chi + ((long)s * g.V + y) * 12;
        for (int al = 0; al < 4; al++) {
          cplx vf[3], vb[3];
          for (int b = 0; b < 3; b++) {
            vf[b] = 0;
            vb[b] = 0;
            for (int be = 0; be < 4; be++) {
              cplx id = al == be ? 1.0 : 0.0;
              cplx gm = PLANT(14) ? -G[mu][al][be] : G[mu][al][be];
              vf[b] += (id - gm) * py[be * 3 + b];
              vb[b] += (id + gm) * px[be * 3 + b];
            }
          }
          for (int b = 0; b < 3; b++)
            for (int a = 0; a < 3; a++) {
              A[b][a] += vf[b] * conj(cx[al * 3 + a]);
              B[b][a] += vb[b] * conj(cy[al * 3 + a]);
            }
        }
      }
      cplx M[3][3];
      for (int b = 0; b < 3; b++)
        for (int a = 0; a < 3; a++) M[b][a] = -0.5 * bs * (A[b][a] + (PLANT(13) ? 0.0 : conj(B[a][b])));
      const cplx* u = U + (x * 4 + mu) * 9;
      cplx X[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
          X[a][b] = 0;
          for (int c = 0; c < 3; c++) X[a][b] += u[a * 3 + c] * M[c][b];
        }
      cplx tr = 0;
      for (int a = 0; a < 3; a++) tr += X[a][a] - conj(X[a][a]);
      cplx* f = F + (x * 4 + mu) * 9;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) f[a * 3 + b] = 0.5 * (X[a][b] - conj(X[b][a])) - (a == b ? tr / 6.0 : 0.0);
    }
  }
  return 0;
}

/* one right-hand side: out = op(in), full-lattice 5D fields */
int oracle_apply(const int dims[4], int bc_t, const cplx* U, int Ns, double m0, const double* omega,
                 double mu, int op, const cplx* in, cplx* out) {
  ctx_t c;
  if (ctx_init(&c, dims, bc_t, U, Ns, m0, omega, mu)) {
    ctx_free(&c);
    return -1;
  }
  int rc = apply_op(&c, op, in, out);
  ctx_free(&c);
  return rc;
}

/* Textbook conjugate gradient on N = S_e^dag S_e (Hestenes-Stiefel):
 *   r = f - N y, p = r;  repeat: alpha = |r|^2 / <p, N p>, y += alpha p,
 *   r -= alpha N p, beta = |r_new|^2 / |r|^2, p = r + beta p,
 * stopping when |r| <= tol |f|.  Returns iterations, or -1 on non-convergence. */
static int cg_normal(const ctx_t* c, const cplx* f, cplx* y, double tol, int maxiter,
                     double* relres) {
  long n = c->n5;
  cplx* r = malloc(sizeof(cplx) * n);
  cplx* p = malloc(sizeof(cplx) * n);
  cplx* Np = malloc(sizeof(cplx) * n);
  op_schur_normal(c, y, Np);
  for (long i = 0; i < n; i++) r[i] = f[i] - Np[i];
  memcpy(p, r, sizeof(cplx) * n);
  double ff = vnorm2(n, f);
  double rr = vnorm2(n, r);
  int k = 0;
  while (k < maxiter && rr > tol * tol * ff) {
    op_schur_normal(c, p, Np);
    double pNp = creal(vdot(n, p, Np));
    double alpha = rr / pNp;
    for (long i = 0; i < n; i++) {
      y[i] += alpha * p[i];
      r[i] -= alpha * Np[i];
    }
    double rr_new = vnorm2(n, r);
    double beta = rr_new / rr;
    rr = rr_new;
    for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
    k++;
  }
  /* true residual */
  op_schur_normal(c, y, Np);
  for (long i = 0; i < n; i++) r[i] = f[i] - Np[i];
  *relres = sqrt(vnorm2(n, r) / ff);
  free(r); free(p); free(Np);
  return rr <= tol * tol * ff ? k : -1;
}

/* Solve with one right-hand side.
 * mode EO_NORMAL: S_e^dag S_e y = b_e (even sites of b), x_e = y, x_o = 0.
 * mode FULL:      D x = b through the even-odd Schur complement:
 *   b' = omega^{-1} b, phi_e = A^{-1}(b'_e - W_eo A^{-1} b'_o),
 *   S_e^dag S_e y_e = S_e^dag phi_e (CG),  y_o = A^{-1}(b'_o - W_oe y_e),
 *   x = (1 + L)^{-1} y.
 * x holds the initial guess on entry (its even sites, as y_e in FULL mode
 * expressed as x; pass zeros for a cold start) and the solution on exit.
 * Returns the iteration count, or -1 when maxiter is reached. */
int oracle_solve(const int dims[4], int bc_t, const cplx* U, int Ns, double m0, const double* omega,
                 double mu, int mode, double tol, int maxiter, const cplx* b, cplx* x,
                 double* relres, double* full_relres) {
  ctx_t c;
  if (ctx_init(&c, dims, bc_t, U, Ns, m0, omega, mu)) {
    ctx_free(&c);
    return -2;
  }
  long n = c.n5, vs = c.g.V * 12;
  int iters;
  *full_relres = -1;
  if (mode == OR_SOLVE_EO_NORMAL) {
    cplx* f = malloc(sizeof(cplx) * n);
    memcpy(f, b, sizeof(cplx) * n);
    mask_parity(&c.g, Ns, f, 1);
    mask_parity(&c.g, Ns, x, 1);
    iters = cg_normal(&c, f, x, tol, maxiter, relres);
    free(f);
  } else {
    cplx* bp = malloc(sizeof(cplx) * n);
    cplx* t1 = malloc(sizeof(cplx) * n);
    cplx* t2 = malloc(sizeof(cplx) * n);
    cplx* phi = malloc(sizeof(cplx) * n);
    cplx* f = malloc(sizeof(cplx) * n);
    cplx* y = malloc(sizeof(cplx) * n);
    for (long i = 0; i < n; i++) bp[i] = b[i] / c.omega[i / vs];
    /* phi_e */
    apply_m5(&c.g, Ns, c.Ainv, bp, t1, 1);       /* A^{-1} b'_o           */
    hop5(&c, 0, t1, t2, 0, 1);                   /* W_eo A^{-1} b'_o      */
    for (long i = 0; i < n; i++) t1[i] = bp[i] - t2[i];
    apply_m5(&c.g, Ns, c.Ainv, t1, phi, 0);      /* A^{-1}(b'_e - ...)    */
    op_schur_dag(&c, phi, f);
    /* initial guess: y_e = ((1 + L) x)_e */
    int m = 4 * Ns;
    cplx* onePlusL = malloc(sizeof(cplx) * m * m);
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) onePlusL[i * m + j] = (i == j ? 1.0 : 0.0) + c.L[i * m + j];
    apply_m5(&c.g, Ns, onePlusL, x, y, 0);
    iters = cg_normal(&c, f, y, tol, maxiter, relres);
    /* y_o */
    hop5(&c, 0, y, t1, 1, 0);                    /* W_oe y_e              */
    for (long i = 0; i < n; i++) t2[i] = bp[i] - t1[i];
    apply_m5(&c.g, Ns, c.Ainv, t2, t1, 1);       /* y_o (odd sites)       */
    for (long i = 0; i < n; i++) y[i] += t1[i];
    apply_m5(&c.g, Ns, c.onePlusLinv, y, x, -1); /* x = (1 + L)^{-1} y    */
    /* full-system residual |b - D x| / |b| */
    op_D(&c, x, t1);
    for (long i = 0; i < n; i++) t1[i] = b[i] - t1[i];
    *full_relres = sqrt(vnorm2(n, t1) / vnorm2(n, b));
    free(bp); free(t1); free(t2); free(phi); free(f); free(y); free(onePlusL);
  }
  ctx_free(&c);
  return iters;
}

/* |f - N y| / |f| with N = S_e^dag S_e, f and y on even sites: the true
 * residual of a solution computed elsewhere. */
double oracle_normal_residual(const int dims[4], int bc_t, const cplx* U, int Ns, double m0,
                              const double* omega, double mu, const cplx* f, const cplx* y) {
  ctx_t c;
  ctx_init(&c, dims, bc_t, U, Ns, m0, omega, mu);
  long n = c.n5;
  cplx* fe = malloc(sizeof(cplx) * n);
  cplx* ye = malloc(sizeof(cplx) * n);
  cplx* t = malloc(sizeof(cplx) * n);
  memcpy(fe, f, sizeof(cplx) * n);
  memcpy(ye, y, sizeof(cplx) * n);
  mask_parity(&c.g, c.Ns, fe, 1);
  mask_parity(&c.g, c.Ns, ye, 1);
  op_schur_normal(&c, ye, t);
  for (long i = 0; i < n; i++) t[i] = PLANT(11) ? fe[i] + t[i] : fe[i] - t[i];
  double r = sqrt(vnorm2(n, t) / vnorm2(n, fe));
  free(fe); free(ye); free(t);
  ctx_free(&c);
  return r;
}
