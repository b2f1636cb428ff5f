/*
 * emg_oracle.c -- plain, slow, FP64 CPU oracle for the node-based
 * finite-difference elasticity operator of Runnels, Agrawal, Zhang and
 * Almgren (arXiv 2001.04789) and for the pieces of its geometric multigrid
 * cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Everything is written as the plain definition: every row sums over the
 * full fourth-order tensor C_ijkl (expanded from its stored form at every
 * use), derivatives are evaluated one finite difference at a time, and no
 * loop is blocked, fused or reordered.  OpenMP only splits the loop over
 * nodes; each node's value is computed exactly as in the serial loop.
 *
 * Discrete system (Sec. 2.1, eqs. elastic_int / elastic_b1 / elastic_b2, and
 * the product-rule split of Sec. 2.1.1):
 *   interior rows   D_H(u)_i = sum_jkl  d_j(C_ijkl) d_l(u_k) + C_ijkl d_jl(u_k)
 *   traction rows   sum over the traction faces f of the node of
 *                   sum_jkl C_ijkl dhat_l(u_k) n^f_j
 *   Dirichlet rows  u_i
 *   Neumann rows    sum over the Neumann faces f of the node of
 *                   n^f_a dhat_a(u_i), a the normal axis of f (eq. elastic_b3)
 * d_j is the central difference, d_jj the 3-point second difference, d_jl
 * (j != l) the 4-corner mixed difference, dhat_l the 3-point one-sided
 * difference pointing into the domain along an axis on whose end the node
 * sits (central otherwise).  Periodic axes wrap and carry no boundary rows.
 * Readings of points the paper leaves open are listed in the design notes
 * of the repository (boundary-row form at edges, Dirichlet precedence,
 * restriction by row class, coarse moduli by full weighting).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_DIRICHLET = 0, ORA_TRACTION = 1, ORA_PERIODIC = 2, ORA_NEUMANN = 3 };
enum { ORA_ISO = 0, ORA_ANISO = 1 };
enum { ROW_INTERIOR = 0, ROW_TRACTION = 1, ROW_DIRICHLET = 2, ROW_NEUMANN = 3 };

typedef struct {
  int dim;       /* 2 or 3 */
  int m[3];      /* stored (unique) nodes per axis; periodic axes hold n-1; m[2] = 1 in 2D */
  double h[3];   /* node spacing per axis */
  int bc[6];     /* face 2a = low end of axis a, 2a+1 = high end */
  int kind;      /* ORA_ISO: (lambda, mu) per node; ORA_ANISO: Voigt upper triangle per node */
} ora_grid;

static long nnodes(const ora_grid *g) { return (long)g->m[0] * g->m[1] * g->m[2]; }

static int periodic(const ora_grid *g, int a) { return g->bc[2 * a] == ORA_PERIODIC; }

/* Index of node p shifted by offsets o; periodic axes wrap. */
static long node_at(const ora_grid *g, const int p[3], const int o[3]) {
  int c[3];
  for (int a = 0; a < 3; a++) {
    c[a] = p[a] + o[a];
    if (a < g->dim && periodic(g, a)) {
      c[a] %= g->m[a];
      if (c[a] < 0) c[a] += g->m[a];
    }
  }
  return ((long)c[2] * g->m[1] + c[1]) * g->m[0] + c[0];
}

static void coords(const ora_grid *g, long n, int p[3]) {
  p[0] = (int)(n % g->m[0]);
  p[1] = (int)((n / g->m[0]) % g->m[1]);
  p[2] = (int)(n / ((long)g->m[0] * g->m[1]));
}

/* Voigt slot of the symmetric index pair (i,j).  3D: 11,22,33,23,31,12 ->
 * 0..5 (Sec. 4.3, Voigt stress/strain vectors); 2D plane strain: 11,22,12 -> 0..2. */
static int voigt(int dim, int i, int j) {
  if (i == j) return i;
  if (dim == 2) return 2;
  return 3 + (3 - i - j);
}

/* Position of (I,J) in the row-major upper triangle of an n x n symmetric matrix. */
static int upper(int n, int I, int J) {
  if (I > J) { int t = I; I = J; J = t; }
  return I * n - I * (I - 1) / 2 + (J - I);
}

static int n_moduli(const ora_grid *g) {
  if (g->kind == ORA_ISO) return 2;
  return g->dim == 3 ? 21 : 6;
}

static int kron(int a, int b) { return a == b; }

/* Full stiffness tensor component C_ijkl at node n, expanded from storage. */
static double Cijkl(const ora_grid *g, const double *C, long n, int i, int j, int k, int l) {
  long N = nnodes(g);
  if (g->kind == ORA_ISO) {
    double lam = C[n], mu = C[N + n];
    return lam * kron(i, j) * kron(k, l) + mu * (kron(i, k) * kron(j, l) + kron(i, l) * kron(j, k));
  }
  int nv = g->dim == 3 ? 6 : 3;
  return C[(long)upper(nv, voigt(g->dim, i, j), voigt(g->dim, k, l)) * N + n];
}

/* Symmetric second-order tensor component from its stored Voigt-ordered
 * tensor components (not engineering shears): eps_kl. */
static double sym2(const ora_grid *g, const double *E, long n, int k, int l) {
  return E[(long)voigt(g->dim, k, l) * nnodes(g) + n];
}

static int at_low(const ora_grid *g, const int p[3], int a) { return !periodic(g, a) && p[a] == 0; }
static int at_high(const ora_grid *g, const int p[3], int a) { return !periodic(g, a) && p[a] == g->m[a] - 1; }

/* 1 if p lies on face f (2a = low end of axis a, 2a+1 = high end) */
static int on_face(const ora_grid *g, const int p[3], int f) {
  return (f % 2 == 0) ? at_low(g, p, f / 2) : at_high(g, p, f / 2);
}

/* Row class of node p: a Dirichlet face of the node decides first, then a
 * Neumann face, then a traction face; nodes on no face are interior. */
static int row_class(const ora_grid *g, const int p[3]) {
  int face = 0, neu = 0;
  for (int f = 0; f < 2 * g->dim; f++) {
    if (!on_face(g, p, f)) continue;
    if (g->bc[f] == ORA_DIRICHLET) return ROW_DIRICHLET;
    face = 1;
    if (g->bc[f] == ORA_NEUMANN) neu = 1;
  }
  return neu ? ROW_NEUMANN : (face ? ROW_TRACTION : ROW_INTERIOR);
}

/* ---- finite differences of a stored scalar field f (component already offset) ---- */

static double fval(const ora_grid *g, const double *f, const int p[3], int da, int oa, int db, int ob) {
  int o[3] = {0, 0, 0};
  o[da] += oa;
  o[db] += ob;
  return f[node_at(g, p, o)];
}

/* central first difference along axis a */
static double d1(const ora_grid *g, const double *f, const int p[3], int a) {
  return (fval(g, f, p, a, 1, a, 0) - fval(g, f, p, a, -1, a, 0)) / (2.0 * g->h[a]);
}

/* second difference d_ab: 3-point if a == b, 4-corner mixed otherwise */
static double d2(const ora_grid *g, const double *f, const int p[3], int a, int b) {
  if (a == b)
    return (fval(g, f, p, a, 1, a, 0) - 2.0 * fval(g, f, p, a, 0, a, 0) + fval(g, f, p, a, -1, a, 0)) /
           (g->h[a] * g->h[a]);
  return (fval(g, f, p, a, 1, b, 1) - fval(g, f, p, a, 1, b, -1) - fval(g, f, p, a, -1, b, 1) +
          fval(g, f, p, a, -1, b, -1)) /
         (4.0 * g->h[a] * g->h[b]);
}

/* first difference along a for a boundary row: 3-point one-sided pointing
 * into the domain when p sits on an end of non-periodic axis a, else central */
static double dhat(const ora_grid *g, const double *f, const int p[3], int a) {
  if (at_low(g, p, a))
    return (-3.0 * fval(g, f, p, a, 0, a, 0) + 4.0 * fval(g, f, p, a, 1, a, 0) - fval(g, f, p, a, 2, a, 0)) /
           (2.0 * g->h[a]);
  if (at_high(g, p, a))
    return (3.0 * fval(g, f, p, a, 0, a, 0) - 4.0 * fval(g, f, p, a, -1, a, 0) + fval(g, f, p, a, -2, a, 0)) /
           (2.0 * g->h[a]);
  return d1(g, f, p, a);
}

/* centre coefficient of dhat along a at p (0 for the central difference) */
static double dhat_centre(const ora_grid *g, const int p[3], int a) {
  if (at_low(g, p, a)) return -3.0 / (2.0 * g->h[a]);
  if (at_high(g, p, a)) return 3.0 / (2.0 * g->h[a]);
  return 0.0;
}

/* central difference of the tensor component C_ijkl along axis a */
static double dC(const ora_grid *g, const double *C, const int p[3], int a, int i, int j, int k, int l) {
  int op[3] = {0, 0, 0}, om[3] = {0, 0, 0};
  op[a] = 1;
  om[a] = -1;
  return (Cijkl(g, C, node_at(g, p, op), i, j, k, l) - Cijkl(g, C, node_at(g, p, om), i, j, k, l)) /
         (2.0 * g->h[a]);
}

/* central difference of the eigenstrain component eps_kl along axis a */
static double dE(const ora_grid *g, const double *E, const int p[3], int a, int k, int l) {
  int op[3] = {0, 0, 0}, om[3] = {0, 0, 0};
  op[a] = 1;
  om[a] = -1;
  return (sym2(g, E, node_at(g, p, op), k, l) - sym2(g, E, node_at(g, p, om), k, l)) / (2.0 * g->h[a]);
}

/* outward normal component along axis a of the face(s) of p on axis a:
 * -1 on the low end, +1 on the high end, 0 if p is on neither */
static double normal(const ora_grid *g, const int p[3], int a) {
  if (at_low(g, p, a)) return -1.0;
  if (at_high(g, p, a)) return 1.0;
  return 0.0;
}

/* ---- the operator D_H (Sec. 2.1.1 product rule; boundary operators of Sec. 2.1) ---- */

static double row_value(const ora_grid *g, const double *C, const double *u, long n, int i) {
  int p[3];
  coords(g, n, p);
  long N = nnodes(g);
  int d = g->dim;
  int cls = row_class(g, p);
  if (cls == ROW_DIRICHLET) return u[(long)i * N + n];
  double acc = 0.0;
  if (cls == ROW_INTERIOR) {
    for (int j = 0; j < d; j++)
      for (int k = 0; k < d; k++)
        for (int l = 0; l < d; l++) {
          const double *uk = u + (long)k * N;
          acc += dC(g, C, p, j, i, j, k, l) * d1(g, uk, p, l);
          acc += Cijkl(g, C, n, i, j, k, l) * d2(g, uk, p, j, l);
        }
    return acc;
  }
  if (cls == ROW_NEUMANN) {
    /* normal derivative of u_i summed over the node's Neumann faces */
    for (int f = 0; f < 2 * d; f++)
      if (on_face(g, p, f) && g->bc[f] == ORA_NEUMANN)
        acc += normal(g, p, f / 2) * dhat(g, u + (long)i * N, p, f / 2);
    return acc;
  }
  /* traction row: sum over the faces the node lies on */
  for (int a = 0; a < d; a++) {
    double na = normal(g, p, a);
    if (na == 0.0) continue;
    for (int k = 0; k < d; k++)
      for (int l = 0; l < d; l++)
        acc += Cijkl(g, C, n, i, a, k, l) * na * dhat(g, u + (long)k * N, p, l);
  }
  return acc;
}

void ora_apply(const ora_grid *g, const double *C, const double *u, double *out) {
  long N = nnodes(g);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++)
    for (int i = 0; i < g->dim; i++) out[(long)i * N + n] = row_value(g, C, u, n, i);
}

/* Coefficient of u_i at node n in row i of D_H. */
static double diag_value(const ora_grid *g, const double *C, long n, int i) {
  int p[3];
  coords(g, n, p);
  int cls = row_class(g, p);
  if (cls == ROW_DIRICHLET) return 1.0;
  double acc = 0.0;
  if (cls == ROW_INTERIOR) {
    for (int j = 0; j < g->dim; j++) acc += Cijkl(g, C, n, i, j, i, j) * (-2.0 / (g->h[j] * g->h[j]));
    return acc;
  }
  if (cls == ROW_NEUMANN) {
    for (int f = 0; f < 2 * g->dim; f++)
      if (on_face(g, p, f) && g->bc[f] == ORA_NEUMANN) acc += normal(g, p, f / 2) * dhat_centre(g, p, f / 2);
    return acc;
  }
  for (int a = 0; a < g->dim; a++) {
    double na = normal(g, p, a);
    if (na == 0.0) continue;
    for (int l = 0; l < g->dim; l++) acc += Cijkl(g, C, n, i, a, i, l) * na * dhat_centre(g, p, l);
  }
  return acc;
}

void ora_diag(const ora_grid *g, const double *C, double *out) {
  long N = nnodes(g);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++)
    for (int i = 0; i < g->dim; i++) out[(long)i * N + n] = diag_value(g, C, n, i);
}

void ora_row_class(const ora_grid *g, int *out) {
  long N = nnodes(g);
  for (long n = 0; n < N; n++) {
    int p[3];
    coords(g, n, p);
    out[n] = row_class(g, p);
  }
}

/* ---- right-hand side: -(D(0) + b) on interior rows, boundary data on boundary rows ----
 * eps0: tensor components in Voigt order (d(d+1)/2 per node) or NULL;
 * b: d per node or NULL; face[f]: d components per node of face f, stored
 * [comp][z][y][x] with the face's normal axis of extent 1, or NULL (= 0).
 * For Dirichlet faces face[f] holds u0, for traction faces t0, for
 * Neumann faces the prescribed normal derivative du0.                     */
static double face_value(const ora_grid *g, const double *F, const int p[3], int a, int i) {
  if (!F) return 0.0;
  int q[3] = {p[0], p[1], p[2]};
  int fm[3] = {g->m[0], g->m[1], g->m[2]};
  q[a] = 0;
  fm[a] = 1;
  long fn = (long)fm[0] * fm[1] * fm[2];
  return F[(long)i * fn + ((long)q[2] * fm[1] + q[1]) * fm[0] + q[0]];
}

void ora_rhs(const ora_grid *g, const double *C, const double *eps0, const double *b, const double *const face[6],
             double *out) {
  long N = nnodes(g);
  int d = g->dim;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    int p[3];
    coords(g, n, p);
    int cls = row_class(g, p);
    for (int i = 0; i < d; i++) {
      double acc = 0.0;
      if (cls == ROW_DIRICHLET) {
        /* the lowest-numbered Dirichlet face the node lies on supplies u0 */
        for (int f = 0; f < 2 * d; f++) {
          int a = f / 2;
          int on = (f % 2 == 0) ? at_low(g, p, a) : at_high(g, p, a);
          if (on && g->bc[f] == ORA_DIRICHLET) { acc = face_value(g, face[f], p, a, i); break; }
        }
      } else if (cls == ROW_NEUMANN) {
        for (int f = 0; f < 2 * d; f++)
          if (on_face(g, p, f) && g->bc[f] == ORA_NEUMANN) acc += face_value(g, face[f], p, f / 2, i);
      } else if (cls == ROW_INTERIOR) {
        if (b) acc -= b[(long)i * N + n];
        if (eps0)
          for (int j = 0; j < d; j++)
            for (int k = 0; k < d; k++)
              for (int l = 0; l < d; l++)
                acc += dC(g, C, p, j, i, j, k, l) * sym2(g, eps0, n, k, l) +
                       Cijkl(g, C, n, i, j, k, l) * dE(g, eps0, p, j, k, l);
      } else {
        for (int f = 0; f < 2 * d; f++) {
          int a = f / 2;
          int on = (f % 2 == 0) ? at_low(g, p, a) : at_high(g, p, a);
          if (!on) continue;
          double na = (f % 2 == 0) ? -1.0 : 1.0;
          acc += face_value(g, face[f], p, a, i);
          if (eps0)
            for (int k = 0; k < d; k++)
              for (int l = 0; l < d; l++) acc += Cijkl(g, C, n, i, a, k, l) * sym2(g, eps0, n, k, l) * na;
        }
      }
      out[(long)i * N + n] = acc;
    }
  }
}

/* ---- stress sigma_ij = C_ijkl (u_k,l - eps0_kl), Voigt output ---- */
void ora_stress(const ora_grid *g, const double *C, const double *eps0, const double *u, double *out) {
  long N = nnodes(g);
  int d = g->dim;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    int p[3];
    coords(g, n, p);
    for (int i = 0; i < d; i++)
      for (int j = i; j < d; j++) {
        double acc = 0.0;
        for (int k = 0; k < d; k++)
          for (int l = 0; l < d; l++) {
            double strain = dhat(g, u + (long)k * N, p, l);
            if (eps0) strain -= sym2(g, eps0, n, k, l);
            acc += Cijkl(g, C, n, i, j, k, l) * strain;
          }
        out[(long)voigt(d, i, j) * N + n] = acc;
      }
  }
}

/* ---- damped Jacobi sweep and residual (Sec. 3.1 relaxation) ---- */
void ora_residual(const ora_grid *g, const double *C, const double *u, const double *f, double *r) {
  long N = nnodes(g);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++)
    for (int i = 0; i < g->dim; i++) r[(long)i * N + n] = f[(long)i * N + n] - row_value(g, C, u, n, i);
}

void ora_jacobi(const ora_grid *g, const double *C, const double *u, const double *f, double omega, double *out) {
  long N = nnodes(g);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    int p[3];
    coords(g, n, p);
    int dir = row_class(g, p) == ROW_DIRICHLET;
    for (int i = 0; i < g->dim; i++) {
      long q = (long)i * N + n;
      if (dir)
        out[q] = f[q];
      else
        out[q] = u[q] + omega * (f[q] - row_value(g, C, u, n, i)) / diag_value(g, C, n, i);
    }
  }
}

/* ---- transfers between a fine grid gf and the next coarser grid gc (ratio 2) ---- */

/* Full-weighting restriction of a fine residual (Sec. 3.2, tensor product of
 * [1/4, 1/2, 1/4]); along an axis on whose end the coarse node sits only the
 * coincident fine node is taken, so boundary row classes never mix with
 * interior ones; Dirichlet coarse rows get 0. */
void ora_restrict(const ora_grid *gf, const ora_grid *gc, const double *rf, double *fc) {
  long Nf = nnodes(gf), Nc = nnodes(gc);
  int d = gf->dim;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < Nc; n++) {
    int P[3];
    coords(gc, n, P);
    int dir = row_class(gc, P) == ROW_DIRICHLET;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < d; a++)
      if (!(at_low(gc, P, a) || at_high(gc, P, a))) { lo[a] = -1; hi[a] = 1; }
    int pf[3] = {2 * P[0], 2 * P[1], 2 * P[2]};
    for (int i = 0; i < d; i++) {
      double acc = 0.0;
      if (!dir)
        for (int oz = lo[2]; oz <= hi[2]; oz++)
          for (int oy = lo[1]; oy <= hi[1]; oy++)
            for (int ox = lo[0]; ox <= hi[0]; ox++) {
              int o[3] = {ox, oy, oz};
              double w = 1.0;
              for (int a = 0; a < d; a++)
                if (hi[a]) w *= (o[a] == 0) ? 0.5 : 0.25;
              acc += w * rf[(long)i * Nf + node_at(gf, pf, o)];
            }
      fc[(long)i * Nc + n] = acc;
    }
  }
}

/* Bilinear / trilinear interpolation of a coarse correction, added to the
 * fine field (Sec. 3.2); Dirichlet fine rows are left untouched. */
void ora_prolong_add(const ora_grid *gc, const ora_grid *gf, const double *ec, double *uf) {
  long Nf = nnodes(gf), Nc = nnodes(gc);
  int d = gf->dim;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < Nf; n++) {
    int p[3];
    coords(gf, n, p);
    if (row_class(gf, p) == ROW_DIRICHLET) continue;
    int base[3], cnt[3];
    for (int a = 0; a < 3; a++) {
      base[a] = p[a] / 2;
      cnt[a] = (a < d && (p[a] % 2)) ? 2 : 1;
    }
    for (int i = 0; i < d; i++) {
      double acc = 0.0;
      for (int cz = 0; cz < cnt[2]; cz++)
        for (int cy = 0; cy < cnt[1]; cy++)
          for (int cx = 0; cx < cnt[0]; cx++) {
            int o[3] = {cx, cy, cz};
            double w = 1.0;
            for (int a = 0; a < d; a++)
              if (cnt[a] == 2) w *= 0.5;
            acc += w * ec[(long)i * Nc + node_at(gc, base, o)];
          }
      uf[(long)i * Nf + n] += acc;
    }
  }
}

/* Coarse-level moduli: full weighting of every stored component, with
 * injection along an axis on whose end the coarse node sits. */
void ora_coarsen_moduli(const ora_grid *gf, const ora_grid *gc, const double *Cf, double *Cc) {
  long Nf = nnodes(gf), Nc = nnodes(gc);
  int d = gf->dim, nc = n_moduli(gf);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < Nc; n++) {
    int P[3];
    coords(gc, n, P);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < d; a++)
      if (!(at_low(gc, P, a) || at_high(gc, P, a))) { lo[a] = -1; hi[a] = 1; }
    int pf[3] = {2 * P[0], 2 * P[1], 2 * P[2]};
    for (int c = 0; c < nc; c++) {
      double acc = 0.0;
      for (int oz = lo[2]; oz <= hi[2]; oz++)
        for (int oy = lo[1]; oy <= hi[1]; oy++)
          for (int ox = lo[0]; ox <= hi[0]; ox++) {
            int o[3] = {ox, oy, oz};
            double w = 1.0;
            for (int a = 0; a < d; a++)
              if (hi[a]) w *= (o[a] == 0) ? 0.5 : 0.25;
            acc += w * Cf[(long)c * Nf + node_at(gf, pf, o)];
          }
      Cc[(long)c * Nc + n] = acc;
    }
  }
}

/* Squared 2-norm of a d-component field over the non-Dirichlet rows. */
double ora_norm2(const ora_grid *g, const double *r) {
  long N = nnodes(g);
  double s = 0.0;
  for (long n = 0; n < N; n++) {
    int p[3];
    coords(g, n, p);
    if (row_class(g, p) == ROW_DIRICHLET) continue;
    for (int i = 0; i < g->dim; i++) s += r[(long)i * N + n] * r[(long)i * N + n];
  }
  return s;
}
