/*
 * Plain FP64 CPU oracle of the exact model-to-scene matching.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the HIP path.
 *
 * It restates Lombardi, Wolf, Celiktutan and Sankur, "Activity recognition from
 * videos with parallel hypergraph matching on GPUs" (arXiv 1505.00581):
 *   - energy terms: Eq. 1-6 (Section 2), constraints Eq. 7-8 (Section 2.1);
 *   - the chain energy Eq. 9 and the literal BACKWARD recursion of Section 2.2:
 *     alpha_M initialisation (Eq. 11), alpha_i recursion with argmin table
 *     beta_i (Eq. 10), the initial search over (z_1, z_2) (Eq. 13) and
 *     backtracking z_i = beta_i(z_{i-1}, z_{i-2}) (Eq. 12);
 *   - each triangle cost is evaluated from its definition with atan2, and the
 *     optimum is re-evaluated with the literal energy (Eq. 1) at the end.
 * Candidate lists per (offset, model point) follow the windowed search rule
 * (a bounded stand-in for the paper's trellis pruning, Sections 3.2 and 3.4):
 * nodes within W frames of the shifted model frame, first K by
 * (|frame difference|, node id), stored in ascending node order.
 *
 * Dummy assignments (Eq. 2): when enabled, every model point may also take the
 * dummy value z_i = epsilon (node id -2 in assignments) at the cost U = W^d.
 * READING (the paper defines only U for a dummy): each term of D is evaluated
 * where its points exist -- Delta(p, q) only when z_p and z_q are both scene
 * points, D^g only when all three are -- and causality and closeness apply
 * to consecutive points that are both scene points.
 *
 * Indices are 0-based: model points 0..M-1, the triangle ending at point i
 * (i >= 2) is (i, i-1, i-2).  Everything is FP64; float inputs are upcast.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846
/* bits of the `readings` argument: alternative readings of the paper */
#define ORACLE_SPAN 1     /* closeness as the span of each triangle (Eq. 14) */
#define ORACLE_UNSIGNED 2 /* unsigned triangle angles (Eq. 6) */
#define ORACLE_NODE 4     /* causality by scene node order (Eq. 7 alternative) */
#define ORACLE_EPS (-2) /* the dummy value epsilon in assignments */

typedef struct {
  int32_t M, S, F, dim;
  const float *mxy, *mdesc, *sxy, *sdesc;
  const int32_t *mt, *st;
  double lambda1, lambda2, lambda3;
  int32_t T, W, K, k_density;
  int32_t dummy; /* dummy assignments enabled */
  double wd;     /* W^d, the unary cost of a dummy (Eq. 2) */
  int32_t span;  /* closeness as the span of each triangle (see triple_ok) */
  int32_t uns;   /* unsigned triangle angles (see triangle_cost) */
  int32_t node;  /* causality by node order (see pair_ok) */
} problem;

/* Oriented angle at vertex b of triangle (a, b, c), ray b->a to ray b->c;
 * 0 when a side has zero length (Eq. 6, reading: oriented image-plane angle). */
static double ang(double ax, double ay, double bx, double by, double cx, double cy) {
  double ux = ax - bx, uy = ay - by, vx = cx - bx, vy = cy - by;
  if ((ux == 0.0 && uy == 0.0) || (vx == 0.0 && vy == 0.0)) return 0.0;
  return atan2(ux * vy - uy * vx, ux * vx + uy * vy);
}

/* Difference on the circle (Eq. 6). */
static double wrap(double x) { return x - 2.0 * ORACLE_PI * nearbyint(x / (2.0 * ORACLE_PI)); }

/* Causality (Eq. 7) and temporal closeness (Eq. 8) for consecutive points. */
static int admissible(int32_t tp_prev, int32_t tp_cur, int32_t T) {
  if (!(tp_prev < tp_cur)) return 0;
  return T <= 0 || tp_cur - tp_prev < T;
}

/* Delta(p,q) = |(t(p) - t(q)) - (t'(z_p) - t'(z_q))| (Eq. 5). */
static double delta(int32_t tp, int32_t tq, int32_t sp, int32_t sq) {
  long d = ((long)tp - (long)tq) - ((long)sp - (long)sq);
  return (double)(d < 0 ? -d : d);
}

/* A consecutive pair (z_{i-1}, z_i) is allowed: admissible, or a dummy on
 * either side.  Under the span reading only causality binds the pair. */
static int pair_ok(const problem* p, int32_t zprev, int32_t zcur) {
  if (zprev == ORACLE_EPS || zcur == ORACLE_EPS) return 1;
  /* READING (node order): z_{i-1} < z_i as scene node ids, which in a scene
   * sorted by frame allows equal frames; closeness as Eq. 8 */
  if (p->node) return zprev < zcur && (p->T <= 0 || p->st[zcur] - p->st[zprev] < p->T);
  if (p->span) return p->st[zprev] < p->st[zcur];
  return admissible(p->st[zprev], p->st[zcur], p->T);
}

/* READING (span form of temporal closeness, from the loop bounds of Section
 * 3.4, Eq. 14): the first and last scene frames of a triangle (z_{i-2},
 * z_{i-1}, z_i) lie less than T apart.  Always true in the pairwise reading
 * (Eq. 8), and for T <= 0. */
static int triple_ok(const problem* p, int32_t zk, int32_t zi) {
  if (!p->span || p->T <= 0) return 1;
  return p->st[zi] - p->st[zk] < p->T;
}

/* A pair that can sit in an admissible assignment, for the work counts: the
 * pairwise constraints, or under the span reading causality with a gap of at
 * most T - 2 (a triangle holding the pair spans at least one more frame). */
static int cell_ok(const problem* p, int32_t zprev, int32_t zcur) {
  if (p->node) return pair_ok(p, zprev, zcur);
  if (!p->span) return admissible(p->st[zprev], p->st[zcur], p->T);
  if (!(p->st[zprev] < p->st[zcur])) return 0;
  return p->T <= 0 || p->st[zcur] - p->st[zprev] <= p->T - 2;
}

/* D(z_i, z_{i-1}, z_{i-2}) = D^t + lambda3 * D^g (Eq. 3, 4, 6); with dummies,
 * each Delta needs both of its points and D^g all three. */
static double triangle_cost(const problem* p, int i, int32_t zi, int32_t zj, int32_t zk) {
  int j = i - 1, k = i - 2;
  double dt = 0.0;
  if (zi != ORACLE_EPS && zj != ORACLE_EPS) dt += delta(p->mt[i], p->mt[j], p->st[zi], p->st[zj]);
  if (zj != ORACLE_EPS && zk != ORACLE_EPS) dt += delta(p->mt[j], p->mt[k], p->st[zj], p->st[zk]);
  if (zi == ORACLE_EPS || zj == ORACLE_EPS || zk == ORACLE_EPS) return dt;
  const float *m = p->mxy, *s = p->sxy;
  double mid_m = ang(m[2 * i], m[2 * i + 1], m[2 * j], m[2 * j + 1], m[2 * k], m[2 * k + 1]);
  double mid_s = ang(s[2 * zi], s[2 * zi + 1], s[2 * zj], s[2 * zj + 1], s[2 * zk], s[2 * zk + 1]);
  double end_m = ang(m[2 * j], m[2 * j + 1], m[2 * i], m[2 * i + 1], m[2 * k], m[2 * k + 1]);
  double end_s = ang(s[2 * zj], s[2 * zj + 1], s[2 * zi], s[2 * zi + 1], s[2 * zk], s[2 * zk + 1]);
  if (p->uns) {
    /* READING (unsigned angles): the magnitudes of the oriented angles, so a
     * triangle and its mirror image have the same angles */
    mid_m = fabs(mid_m); mid_s = fabs(mid_s); end_m = fabs(end_m); end_s = fabs(end_s);
  }
  double d1 = wrap(mid_m - mid_s), d2 = wrap(end_m - end_s);
  return dt + p->lambda3 * sqrt(d1 * d1 + d2 * d2);
}

/* U(z_i) = ||f_i - f'_{z_i}|| (Eq. 2), squares summed in index order; W^d
 * for the dummy. */
static double unary(const problem* p, int i, int32_t n) {
  if (n == ORACLE_EPS) return p->wd;
  double s = 0.0;
  for (int d = 0; d < p->dim; ++d) {
    double v = (double)p->mdesc[(size_t)i * p->dim + d] - (double)p->sdesc[(size_t)n * p->dim + d];
    s += v * v;
  }
  return sqrt(s);
}

/* E(z) of Eq. 1 / Eq. 9 for a full assignment; +inf if a consecutive pair is
 * inadmissible (or z holds -1, or a dummy while dummies are off).  If eu is
 * non-null it receives lambda1 * sum U. */
double oracle_energy(const problem* p, const int32_t* z, double* eu) {
  for (int i = 0; i < p->M; ++i)
    if (z[i] == -1 || (z[i] == ORACLE_EPS && !p->dummy) || (i > 0 && !pair_ok(p, z[i - 1], z[i])) ||
        (i > 1 && !triple_ok(p, z[i - 2], z[i]))) {
      if (eu) *eu = INFINITY;
      return INFINITY;
    }
  double su = 0.0, sd = 0.0;
  for (int i = 0; i < p->M; ++i) su += unary(p, i, z[i]);
  for (int i = 2; i < p->M; ++i) sd += triangle_cost(p, i, z[i], z[i - 1], z[i - 2]);
  if (eu) *eu = p->lambda1 * su;
  return p->lambda1 * su + p->lambda2 * sd;
}

/* ---- candidate lists ---------------------------------------------------- */

static int32_t lower_bound_t(const int32_t* st, int32_t S, int32_t f) {
  int32_t lo = 0, hi = S;
  while (lo < hi) { int32_t mid = lo + (hi - lo) / 2; if (st[mid] < f) lo = mid + 1; else hi = mid; }
  return lo;
}

static int32_t density_k(const problem* p, int32_t f) {
  int32_t rho = lower_bound_t(p->st, p->S, f + 2) - lower_bound_t(p->st, p->S, f - 1);
  int32_t num = 56 * rho - 1170, k;
  k = num >= 0 ? num / 60 : -((-num + 59) / 60); /* floor division */
  if (k < 8) k = 8;
  if (k > 64) k = 64;
  if (k > p->K) k = p->K;
  return k;
}

typedef struct { int32_t key, node; } keyed;
static int cmp_keyed(const void* a, const void* b) {
  const keyed *x = (const keyed*)a, *y = (const keyed*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->node < y->node ? -1 : (x->node > y->node);
}
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return x < y ? -1 : (x > y);
}

/* Writes up to K node ids (ascending) into out; returns the count. */
static int32_t build_candidates(const problem* p, int32_t tau, int i, int32_t* out, keyed* tmp) {
  int32_t f = tau + p->mt[i] - p->mt[0];
  int32_t lo = lower_bound_t(p->st, p->S, f - p->W);
  int32_t hi = lower_bound_t(p->st, p->S, f + p->W + 1);
  int32_t n = 0;
  for (int32_t v = lo; v < hi; ++v) {
    int32_t d = p->st[v] - f;
    tmp[n].key = d < 0 ? -d : d;
    tmp[n].node = v;
    ++n;
  }
  qsort(tmp, (size_t)n, sizeof(keyed), cmp_keyed);
  int32_t k = p->k_density ? density_k(p, f) : p->K;
  if (n > k) n = k;
  for (int32_t a = 0; a < n; ++a) out[a] = tmp[a].node;
  qsort(out, (size_t)n, sizeof(int32_t), cmp_i32);
  return n;
}

int32_t oracle_candidates(const problem* p, int32_t tau, int32_t i, int32_t* out) {
  keyed* tmp = (keyed*)malloc(sizeof(keyed) * (size_t)(p->S > 0 ? p->S : 1));
  int32_t n = build_candidates(p, tau, i, out, tmp);
  free(tmp);
  return n;
}

/* ---- the literal backward recursion (Section 2.2) ------------------------- */

/* counts[0..3] (nullable): dense cells, feasible cells, dense relaxations, feasible
 * relaxations.  A cell is a state pair of consecutive points (a_{i-1}, a_i);
 * a relaxation is a triple (a_{i-2}, a_{i-1}, a_i); "feasible" means every
 * consecutive pair in it is admissible. */
static int match_one(const problem* p, int32_t tau, const int32_t* given, const int32_t* given_cnt,
                     double* energy, double* energy_u, int32_t* assign, long long* counts) {
  const int M = p->M, K = p->K;
  /* States of point i: its cnt[i] candidates, then the dummy when enabled. */
  const int KS = K + 1;
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)M * K);
  int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  int32_t* nst = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  keyed* tmp = (keyed*)malloc(sizeof(keyed) * (size_t)(p->S > 0 ? p->S : 1));
  double* u = (double*)malloc(sizeof(double) * (size_t)M * KS);
  /* alpha_i(z_{i-1}, z_{i-2}) and beta_i for i = 2..M-1: [a_{i-1}][a_{i-2}] */
  double* alpha = (double*)malloc(sizeof(double) * (size_t)M * KS * KS);
  int32_t* beta = (int32_t*)malloc(sizeof(int32_t) * (size_t)M * KS * KS);
  int32_t* z = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  int rc = 0;

  int empty = 0;
  for (int i = 0; i < M; ++i) {
    if (given) { /* caller's lists, [M][K] with counts [M] */
      cnt[i] = given_cnt[i];
      memcpy(cand + (size_t)i * K, given + (size_t)i * K, sizeof(int32_t) * (size_t)cnt[i]);
    } else {
      cnt[i] = build_candidates(p, tau, i, cand + (size_t)i * K, tmp);
    }
    nst[i] = cnt[i] + (p->dummy ? 1 : 0);
    if (nst[i] == 0) empty = 1;
  }
#define NODE(i, a) ((a) < cnt[i] ? cand[(size_t)(i) * K + (a)] : ORACLE_EPS)
  /* Unary look-up table (Section 3.3): U of every (point, state), lambda1 absorbed. */
  for (int i = 0; i < M; ++i)
    for (int a = 0; a < nst[i]; ++a) u[(size_t)i * KS + a] = p->lambda1 * unary(p, i, NODE(i, a));

  /* work counts (scene candidates only), when asked for */
  for (int i = 1; counts && i < M; ++i)
    for (int b = 0; b < cnt[i - 1]; ++b)
      for (int a = 0; a < cnt[i]; ++a) {
        counts[0] += 1;
        counts[1] += cell_ok(p, cand[(size_t)(i - 1) * K + b], cand[(size_t)i * K + a]);
      }
  for (int i = 2; counts && i < M; ++i)
    for (int c = 0; c < cnt[i - 2]; ++c)
      for (int b = 0; b < cnt[i - 1]; ++b) {
        const int32_t zk = cand[(size_t)(i - 2) * K + c], zj = cand[(size_t)(i - 1) * K + b];
        int ab = cell_ok(p, zk, zj);
        for (int a = 0; a < cnt[i]; ++a) {
          const int32_t zi = cand[(size_t)i * K + a];
          counts[2] += 1;
          counts[3] += ab && cell_ok(p, zj, zi) && triple_ok(p, zk, zi);
        }
      }

  if (empty) goto infeasible;

  /* alpha_M (Eq. 11) and alpha_i (Eq. 10), i from the last point down to 2. */
  for (int i = M - 1; i >= 2; --i) {
    for (int aj = 0; aj < nst[i - 1]; ++aj)
      for (int ak = 0; ak < nst[i - 2]; ++ak) {
        const int32_t zj = NODE(i - 1, aj), zk = NODE(i - 2, ak);
        double best = INFINITY;
        int32_t arg = -1;
        if (pair_ok(p, zk, zj)) {
          for (int ai = 0; ai < nst[i]; ++ai) {
            const int32_t zi = NODE(i, ai);
            if (!pair_ok(p, zj, zi) || !triple_ok(p, zk, zi)) continue;
            double v = u[(size_t)i * KS + ai] + p->lambda2 * triangle_cost(p, i, zi, zj, zk);
            if (i < M - 1) v += alpha[((size_t)(i + 1) * KS + ai) * KS + aj];
            if (v < best) { best = v; arg = ai; }
          }
        }
        alpha[((size_t)i * KS + aj) * KS + ak] = best;
        beta[((size_t)i * KS + aj) * KS + ak] = arg;
      }
  }
  /* Initial search for (z_1, z_2) (Eq. 13): first lexicographic argmin over
   * (a_1, a_2) in that order. */
  {
    double best = INFINITY;
    int32_t b0 = -1, b1 = -1;
    for (int a0 = 0; a0 < nst[0]; ++a0)
      for (int a1 = 0; a1 < nst[1]; ++a1) {
        double v = u[a0] + u[(size_t)KS + a1] + alpha[((size_t)2 * KS + a1) * KS + a0];
        if (v < best) { best = v; b0 = a0; b1 = a1; }
      }
    if (!(best < INFINITY)) goto infeasible;
    /* Backtracking (Eq. 12). */
    int32_t a_prev2 = b0, a_prev1 = b1;
    z[0] = NODE(0, b0);
    z[1] = NODE(1, b1);
    for (int i = 2; i < M; ++i) {
      int32_t ai = beta[((size_t)i * KS + a_prev1) * KS + a_prev2];
      z[i] = NODE(i, ai);
      a_prev2 = a_prev1;
      a_prev1 = ai;
    }
#undef NODE
    double eu = 0.0;
    double e = oracle_energy(p, z, &eu);
    /* The recursion's optimum must equal the literal energy of its argmin. */
    if (!(fabs(e - best) <= 1e-12 * fmax(1.0, fabs(e)))) rc = -5;
    *energy = e;
    if (energy_u) *energy_u = eu;
    for (int i = 0; i < M; ++i) assign[i] = z[i];
  }
  goto done;

infeasible:
  *energy = INFINITY;
  if (energy_u) *energy_u = INFINITY;
  for (int i = 0; i < M; ++i) assign[i] = -1;
done:
  free(cand); free(cnt); free(nst); free(tmp); free(u); free(alpha); free(beta); free(z);
  return rc;
}

static problem make_problem(int32_t M, const float* mxy, const int32_t* mt, const float* mdesc,
                            int32_t S, int32_t F, const float* sxy, const int32_t* st, const float* sdesc,
                            int32_t dim, double l1, double l2, double l3, int32_t T, int32_t W, int32_t K,
                            int32_t k_density, int32_t dummy, double wd, int32_t readings) {
  problem p;
  p.M = M; p.S = S; p.F = F; p.dim = dim;
  p.mxy = mxy; p.mt = mt; p.mdesc = mdesc; p.sxy = sxy; p.st = st; p.sdesc = sdesc;
  p.lambda1 = l1; p.lambda2 = l2; p.lambda3 = l3; p.T = T; p.W = W; p.K = K; p.k_density = k_density;
  p.dummy = dummy; p.wd = wd;
  p.span = readings & ORACLE_SPAN;
  p.uns = (readings & ORACLE_UNSIGNED) != 0;
  p.node = (readings & ORACLE_NODE) != 0;
  return p;
}

/* Exact matching at offsets taus[0..n_tau-1]: energy [n_tau], energy_u [n_tau]
 * (nullable), assign [n_tau*M] (-1 rows if infeasible, -2 for a dummy),
 * counts[4] totals.  dummy != 0 enables dummy assignments of cost wd.
 * Returns 0, or -5 if a re-evaluated optimum disagreed with the recursion. */
int oracle_match(int32_t M, const float* mxy, const int32_t* mt, const float* mdesc,
                 int32_t S, int32_t F, const float* sxy, const int32_t* st, const float* sdesc,
                 int32_t dim, double l1, double l2, double l3, int32_t T, int32_t readings, int32_t W, int32_t K,
                 int32_t k_density, int32_t dummy, double wd, const int32_t* taus, int32_t n_tau,
                 double* energy, double* energy_u, int32_t* assign, long long* counts, int32_t n_threads) {
  problem p = make_problem(M, mxy, mt, mdesc, S, F, sxy, st, sdesc, dim, l1, l2, l3, T, W, K, k_density,
                           dummy, wd, readings);
  long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2, c3) reduction(min : rc)
  for (int32_t j = 0; j < n_tau; ++j) {
    long long c[4] = {0, 0, 0, 0};
    int r = match_one(&p, taus[j], NULL, NULL, energy + j, energy_u ? energy_u + j : NULL, assign + (size_t)j * M, c);
    c0 += c[0]; c1 += c[1]; c2 += c[2]; c3 += c[3];
    if (r < rc) rc = r;
  }
  if (counts) { counts[0] = c0; counts[1] = c1; counts[2] = c2; counts[3] = c3; }
  return rc;
}

/* The same recursion on caller-given candidate lists: lists [n_tau][M][K]
 * (ascending node ids, any subset of the scene), counts [n_tau][M] <= K.  The
 * offsets matter only through the lists.  Returns as oracle_match. */
int oracle_match_lists(int32_t M, const float* mxy, const int32_t* mt, const float* mdesc,
                       int32_t S, int32_t F, const float* sxy, const int32_t* st, const float* sdesc,
                       int32_t dim, double l1, double l2, double l3, int32_t T, int32_t readings, int32_t K,
                       int32_t dummy, double wd, const int32_t* lists, const int32_t* counts_in,
                       int32_t n_tau, double* energy, double* energy_u, int32_t* assign, int32_t n_threads) {
  problem p = make_problem(M, mxy, mt, mdesc, S, F, sxy, st, sdesc, dim, l1, l2, l3, T, 0, K, 0, dummy, wd,
                           readings);
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc)
  for (int32_t j = 0; j < n_tau; ++j) {
    int r = match_one(&p, 0, lists + (size_t)j * M * K, counts_in + (size_t)j * M, energy + j,
                      energy_u ? energy_u + j : NULL, assign + (size_t)j * M, NULL);
    if (r < rc) rc = r;
  }
  return rc;
}

/* E(z) for n assignments z [n*M] (Eq. 1; -2 = dummy when dummy != 0);
 * energy_u nullable. */
void oracle_energies(int32_t M, const float* mxy, const int32_t* mt, const float* mdesc,
                     int32_t S, int32_t F, const float* sxy, const int32_t* st, const float* sdesc,
                     int32_t dim, double l1, double l2, double l3, int32_t T, int32_t readings, int32_t dummy,
                     double wd, const int32_t* z, int32_t n, double* energy, double* energy_u) {
  problem p = make_problem(M, mxy, mt, mdesc, S, F, sxy, st, sdesc, dim, l1, l2, l3, T, 0, 1, 0, dummy, wd,
                           readings);
  for (int32_t j = 0; j < n; ++j)
    energy[j] = oracle_energy(&p, z + (size_t)j * M, energy_u ? energy_u + j : NULL);
}

/* Candidate list of point i at offset tau; out must hold K entries. */
int32_t oracle_candidate_list(int32_t M, const int32_t* mt, int32_t S, const int32_t* st,
                              int32_t W, int32_t K, int32_t k_density, int32_t tau, int32_t i,
                              int32_t* out) {
  problem p = make_problem(M, NULL, mt, NULL, S, 0, NULL, st, NULL, 0, 0, 0, 0, 0, W, K, k_density, 0, 0.0, 0);
  return oracle_candidates(&p, tau, i, out);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
