/* The C ABI (include/emg.h) driven from plain C, with no Python in between:
 * a context; single-level FP64 / mixed (one and two FP32 cycles per
 * refinement step) / F-cycle solves with a warm start;
 * the autotuner (tile shapes of every level) and a solve on its plan;
 * displacement, stress and von Mises read-back; a ragged batch of three
 * problems; a three-level AMR problem in both precisions; a server taking
 * twelve requests of two sizes through three slots; an invalid domain.
 * Data are smooth synthetic fields; the checks are the status codes and
 * convergence.  Build against the in-tree library:
 *
 *   clang++ -O1 -g -I include -x c++ -c tests/native/abi_check.c -o abi_check.o
 *   clang++ abi_check.o -L paper_2001_04789_amd -l:libemg.so -L/opt/rocm/lib -lamdhip64 \
 *     -Wl,-rpath,<repo>/paper_2001_04789_amd -o abi_check
 *
 * Exit status 0 when every call behaves.  For a sanitizer run, compile
 * paper_2001_04789_amd/csrc/emg.hip with hipcc -c and -Xarch_host
 * -fsanitize=address instead of linking libemg.so, build this file and link
 * with clang++ -fsanitize=address, and run with ASAN_OPTIONS=detect_leaks=0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "emg.h"

static int failures = 0;

#define CHECK(call, want)                                                                       \
  do {                                                                                          \
    emg_status s_ = (call);                                                                     \
    if (s_ != (want)) {                                                                         \
      fprintf(stderr, "FAIL %s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #call, (int)s_,          \
              emg_last_error());                                                                \
      failures++;                                                                               \
    }                                                                                           \
  } while (0)

/* stored nodes per axis */
static void stored(const emg_domain *d, int64_t m[3]) {
  for (int a = 0; a < 3; a++) {
    const int per = a < d->dim && d->bc[2 * a] == EMG_BC_PERIODIC;
    m[a] = a < d->dim ? d->n[a] - per : 1;
  }
}

/* isotropic or anisotropic moduli varying smoothly over the grid */
static double *moduli(const emg_domain *d, const int64_t m[3]) {
  const int nc = d->kind == EMG_MOD_ISO ? 2 : (d->dim == 3 ? 21 : 6);
  const int64_t N = m[0] * m[1] * m[2];
  double *C = (double *)calloc((size_t)nc * N, sizeof(double));
  for (int64_t n = 0; n < N; n++) {
    const double x = (double)(n % m[0]) / m[0], y = (double)((n / m[0]) % m[1]) / m[1];
    const double lam = 1.5 + 0.3 * sin(6.0 * x), mu = 1.0 + 0.2 * cos(5.0 * y);
    if (d->kind == EMG_MOD_ISO) {
      C[n] = lam;
      C[N + n] = mu;
    } else {
      const int nv = d->dim == 3 ? 6 : 3;
      int c = 0;
      for (int I = 0; I < nv; I++)
        for (int J = I; J < nv; J++, c++) {
          const int normal = d->dim == 3 ? 3 : 2;
          double v = 0.0;
          if (I < normal && J < normal) v = lam + (I == J ? 2.0 * mu : 0.0);
          else if (I == J) v = mu;
          C[(int64_t)c * N + n] = v;
        }
    }
  }
  return C;
}

static emg_problem *make_problem(emg_ctx *ctx, const emg_domain *d) {
  emg_problem *p = NULL;
  CHECK(emg_problem_create(ctx, d, &p), EMG_OK);
  if (!p) return NULL;
  int64_t m[3];
  stored(d, m);
  double *C = moduli(d, m);
  CHECK(emg_set_moduli(p, C, 0), EMG_OK);
  free(C);
  /* displacement 1e-3 along the last axis on its high face, fixed on its low face */
  const int ax = d->dim - 1;
  int64_t fm[3] = {m[0], m[1], m[2]};
  fm[ax] = 1;
  const int64_t fn = fm[0] * fm[1] * fm[2];
  double *face = (double *)calloc((size_t)d->dim * fn, sizeof(double));
  for (int64_t i = 0; i < fn; i++) face[(int64_t)ax * fn + i] = 1e-3;
  CHECK(emg_set_face(p, 2 * ax + 1, face, 0), EMG_OK);
  free(face);
  return p;
}

static emg_domain domain(int dim, int n, int kind, int periodic_xy) {
  emg_domain d;
  memset(&d, 0, sizeof(d));
  d.dim = dim;
  for (int a = 0; a < 3; a++) {
    d.n[a] = a < dim ? n : 1;
    d.lo[a] = 0.0;
    d.hi[a] = 1.0;
  }
  for (int f = 0; f < 6; f++) d.bc[f] = EMG_BC_TRACTION;
  if (periodic_xy)
    for (int f = 0; f < 2 * (dim - 1); f++) d.bc[f] = EMG_BC_PERIODIC;
  d.bc[2 * (dim - 1)] = EMG_BC_DIRICHLET;
  d.bc[2 * (dim - 1) + 1] = EMG_BC_DIRICHLET;
  if (dim == 2) d.bc[4] = d.bc[5] = EMG_BC_PERIODIC;
  d.kind = kind;
  return d;
}

int main(void) {
  emg_ctx *ctx = NULL;
  CHECK(emg_ctx_create(0, 0, &ctx), EMG_OK);
  if (!ctx) return 1;
  emg_solve_opts o;
  emg_solve_stats st;

  /* single level: FP64, mixed, F-cycle, warm start */
  emg_domain d3 = domain(3, 33, EMG_MOD_ANISO, 1);
  emg_problem *p = make_problem(ctx, &d3);
  emg_default_opts(&o);
  CHECK(emg_solve(p, &o, &st), EMG_OK);
  o.precision = EMG_MIXED;
  CHECK(emg_solve(p, &o, &st), EMG_OK);
  o.inner_cycles = 2;   /* two FP32 cycles per refinement step */
  CHECK(emg_solve(p, &o, &st), EMG_OK);
  if (st.cycles % 2 != 0 || !st.converged) {
    fprintf(stderr, "FAIL inner_cycles=2: %d cycles, converged %d\n", st.cycles, st.converged);
    failures++;
  }
  o.inner_cycles = 1;
  o.cycle = EMG_FCYCLE;
  o.warm_start = 1;
  CHECK(emg_solve(p, &o, &st), EMG_OK);
  int ntuned = -1, nlev = 0;   /* every level has tile-shape variants (no z-march: too narrow) */
  CHECK(emg_num_levels(p, &nlev), EMG_OK);
  CHECK(emg_autotune(p, EMG_FP64, 5, 0, &ntuned), EMG_OK);
  if (ntuned != nlev) {
    fprintf(stderr, "FAIL autotune measured %d of %d levels\n", ntuned, nlev);
    failures++;
  }
  int zm = -1, ts = -1, rs = -1, is = -1;
  CHECK(emg_level_zmarch(p, 0, EMG_FP64, &zm), EMG_OK);
  CHECK(emg_level_tiles(p, 0, EMG_FP64, &ts, &rs, &is), EMG_OK);
  if (zm != 0 || ts < 0 || ts > 3 || rs < 0 || rs > 3 || is < 0 || is > 3) {
    fprintf(stderr, "FAIL tuned plan of level 0: zm %d tiles %d %d %d\n", zm, ts, rs, is);
    failures++;
  }
  int tl = -1;   /* the tuner's choice: 8 x 8 x 9 and the bottom level fused (2) or not (0) */
  CHECK(emg_tail_levels(p, EMG_FP64, &tl), EMG_OK);
  if (tl != 0 && tl != 2) {
    fprintf(stderr, "FAIL fused coarse tail of %d levels, expected 0 or 2\n", tl);
    failures++;
  }
  CHECK(emg_tail_levels(p, 7, &tl), EMG_EINVAL);
  CHECK(emg_solve(p, &o, &st), EMG_OK);   /* a solve on the tuned plan */
  CHECK(emg_autotune(p, EMG_FP64, 0, 0, &ntuned), EMG_EINVAL);
  CHECK(emg_autotune_reset(), EMG_OK);
  int64_t m[3];
  stored(&d3, m);
  double *u = (double *)malloc(sizeof(double) * 3 * m[0] * m[1] * m[2]);
  double *sig = (double *)malloc(sizeof(double) * 6 * m[0] * m[1] * m[2]);
  CHECK(emg_get_displacement(p, u, 0), EMG_OK);
  CHECK(emg_get_stress(p, 0, sig, 0), EMG_OK);
  CHECK(emg_get_von_mises(p, sig, 0), EMG_OK);
  free(u);
  free(sig);

  /* ragged batch: three 3D problems, two sizes and both moduli kinds */
  emg_domain db[3] = {domain(3, 17, EMG_MOD_ISO, 0), domain(3, 33, EMG_MOD_ISO, 1), domain(3, 17, EMG_MOD_ANISO, 1)};
  emg_problem *pb[3];
  for (int i = 0; i < 3; i++) pb[i] = make_problem(ctx, &db[i]);
  emg_solve_stats sb[3];
  emg_default_opts(&o);
  o.precision = EMG_MIXED;
  CHECK(emg_solve_batch(pb, 3, &o, sb), EMG_OK);
  for (int i = 0; i < 3; i++) CHECK(emg_problem_destroy(pb[i]), EMG_OK);

  /* AMR: base 33^3 non-periodic, two nested boxes, FP64 and mixed */
  emg_domain da = domain(3, 33, EMG_MOD_ISO, 0);
  emg_problem *pa = make_problem(ctx, &da);
  /* level 1 as two boxes meeting at y = 32 (their union is one box), level 2 one box */
  const emg_box b1[2] = {{{16, 16, 16}, {48, 32, 48}}, {{16, 32, 16}, {48, 48, 48}}};
  const int64_t lo2[3] = {48, 48, 48}, hi2[3] = {80, 80, 80};
  CHECK(emg_set_level_boxes(pa, 2, b1, 2), EMG_ESTATE);   /* levels are added in order */
  CHECK(emg_set_level_boxes(pa, 1, b1, 2), EMG_OK);
  CHECK(emg_amr_add_level(pa, lo2, hi2), EMG_OK);
  int64_t nvalid = 0;
  CHECK(emg_amr_level_valid(pa, 1, NULL, &nvalid), EMG_OK);
  if (nvalid != 33LL * 33 * 33) {
    fprintf(stderr, "FAIL: level 1 has %lld valid nodes\n", (long long)nvalid);
    failures++;
  }
  for (int k = 1; k <= 2; k++) {
    int64_t bm[3];
    CHECK(emg_amr_level_shape(pa, k, bm), EMG_OK);
    emg_domain db2 = da;
    double *C = moduli(&db2, bm);
    CHECK(emg_amr_set_moduli(pa, k, C, 0), EMG_OK);
    free(C);
  }
  emg_default_opts(&o);
  CHECK(emg_solve(pa, &o, &st), EMG_OK);
  o.precision = EMG_MIXED;
  CHECK(emg_solve(pa, &o, &st), EMG_OK);
  for (int k = 0; k <= 2; k++) {   /* stress on the base grid and on both refined levels */
    int64_t sm[3] = {33, 33, 33};
    if (k) CHECK(emg_amr_level_shape(pa, k, sm), EMG_OK);
    double *sk = (double *)malloc(sizeof(double) * 6 * sm[0] * sm[1] * sm[2]);
    CHECK(emg_get_stress(pa, k, sk, 0), EMG_OK);
    free(sk);
  }
  CHECK(emg_get_stress(pa, 3, sig, 0), EMG_EINVAL);
  CHECK(emg_problem_destroy(pa), EMG_OK);

  /* server: 12 requests of two sizes through 3 slots */
  emg_server *srv = NULL;
  emg_default_opts(&o);
  o.precision = EMG_MIXED;
  o.inner_cycles = 2;
  CHECK(emg_server_create(ctx, 3, &o, &srv), EMG_OK);
  uint64_t tickets[12];
  double *outs[12];
  for (int i = 0; i < 12; i++) {
    emg_domain dr = domain(3, i % 2 ? 33 : 17, EMG_MOD_ANISO, 1);
    int64_t rm[3];
    stored(&dr, rm);
    const int64_t N = rm[0] * rm[1] * rm[2];
    emg_request r;
    memset(&r, 0, sizeof(r));
    r.dom = dr;
    double *C = moduli(&dr, rm);
    r.C = C;
    int64_t fm[3] = {rm[0], rm[1], 1};
    double *face = (double *)calloc((size_t)3 * fm[0] * fm[1], sizeof(double));
    for (int64_t j = 0; j < fm[0] * fm[1]; j++) face[2 * fm[0] * fm[1] + j] = 1e-3;
    r.face[5] = face;
    outs[i] = (double *)malloc(sizeof(double) * 3 * N);
    r.u_out = outs[i];
    CHECK(emg_server_submit(srv, &r, &tickets[i]), EMG_OK);
    free(C);   /* host inputs are copied at submit */
    free(face);
  }
  for (int i = 0; i < 12; i++) {
    emg_ticket_info info;
    CHECK(emg_server_wait(srv, tickets[i], &info), EMG_OK);
    if (info.status != EMG_OK || !info.stats.converged) {
      fprintf(stderr, "FAIL request %d status %d converged %d\n", i, (int)info.status, info.stats.converged);
      failures++;
    }
    free(outs[i]);
  }
  CHECK(emg_server_destroy(srv), EMG_OK);

  /* error paths */
  emg_domain bad = domain(3, 34, EMG_MOD_ISO, 0);
  emg_problem *pbad = NULL;
  CHECK(emg_problem_create(ctx, &bad, &pbad), EMG_EINVAL);
  CHECK(emg_problem_destroy(p), EMG_OK);
  CHECK(emg_ctx_destroy(ctx), EMG_OK);
  printf("abi_check: %d failure(s)\n", failures);
  fflush(stdout);
  return failures ? 1 : 0;
}
