/*
 * ctree.c -- the oracle's tree walk, fitness and forward-mode gradient in C
 * (binary64), for workloads too large for its NumPy implementation.
 *
 * TEST INFRASTRUCTURE ONLY: only the test-suite (through oracle/fast.py) may
 * load this library.  It computes exactly what oracle/tree.py, fitness.py,
 * grad.py and mca.py compute, from the same definitions, row by row instead
 * of vectorised over rows, and shares nothing with the HIP library:
 *   * evaluation is a recursive walk over the heap-ordered genotype (children
 *     of slot i at 2i+1 and 2i+2; a unary operator reads 2i+1; Section 3.1 /
 *     Fig. 1), never over a postfix program;
 *   * operators are the protected ones of the reading in oracle/opset.py
 *     (division and log guarded at GUARD, exp and pow's exponent clamped at
 *     CLAMP), in binary64, every node value rounded to the binary32 range when
 *     asked (|v| beyond it becomes +-inf; precision is not emulated);
 *   * fitness: raw MSE (Eq. 1), the two-pass centred least-squares fit with a
 *     direct residual pass (linear scaling), NMSE (Eq. 2), with the same
 *     degenerate and non-finite rules;
 *   * gradient: forward-mode tangents of every active constant (constants in
 *     post-order), chain-rule products that absorb zeros, the
 *     envelope-theorem sum (2b/N) sum_r (a + b p_r - y_r) dp_r/dc_j (or
 *     (2/N) sum_r (p_r - y_r) dp_r/dc_j), and the term magnitudes gabs;
 *   * Monte-Carlo arithmetic: every operator result (value and tangent)
 *     multiplied by 1 + u eps, u ~ U(-1, 1) from a counter-based generator
 *     (splitmix64 of seed, slot and row) instead of NumPy's stream.
 * Sums are Neumaier-compensated per thread and combined in thread order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ADD = 0, SUB, MUL, DIV, SIN, COS, SQ, SQRT, EXP, LOG, POW };
#define SYM_CONST 32
#define SYM_VAR0 64
#define MAXC 256
#define MAXDEPTH 16

/* the reading of the protected operators (oracle/opset.py) */
static const double GUARD_DEFAULT = 9.99999997475242708e-07; /* binary32 nearest 1e-6 */
static const double CLAMP_DEFAULT = 80.0;
/* smallest magnitude that rounds to infinity in binary32 */
static const double F32_OVERFLOW = 3.4028235677973366e+38;
static const double F32_MAX = 3.4028234663852886e+38;

typedef struct {
  double s, c; /* Neumaier sum and compensation */
} nsum;
static inline void nadd(nsum* a, double v) {
  const double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double nval(const nsum* a) { return a->s + a->c; }

static inline int arity(int g) {
  if (g == ADD || g == SUB || g == MUL || g == DIV || g == POW) return 2;
  if (g >= SIN && g <= LOG) return 1;
  return 0;
}

static inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
/* u in (-1, 1) for (seed, slot, row) */
static inline double mca_u(uint64_t seed, int slot, int64_t row) {
  const uint64_t h = mix64(seed ^ mix64((uint64_t)slot * 0x100000001b3ull ^ mix64((uint64_t)row)));
  return ((double)(h >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

typedef struct {
  const int8_t* genes;
  const double* gc;
  int T, height;
  const float* X;
  int64_t N;
  const float* y;
  int rng_f32, duals, C;
  int cidx[1024]; /* constant ordinal of each slot (post-order), -1 otherwise */
  double guard, clamp, window;
  double eps;
  uint64_t seed;
} Prog;

static inline double clampv(double t, double cl) { return t < -cl ? -cl : (t > cl ? cl : t); }

static inline int near_thr(double v, double thr, double window) {
  const double d = fabs(fabs(v) - thr);
  return d <= window * thr; /* NaN compares false */
}

/* chain-rule product: 0 times anything is 0 */
static inline double chain(double f, double t) { return (f == 0.0 || t == 0.0) ? 0.0 : f * t; }

/* Value of slot i at row r; if P->duals, its tangent in t[0..C) (with *ht = 1
 * when some constant lies below).  `stk` is scratch for the children's
 * tangents.  *near collects whether a decision input lies within the window. */
static double ev(const Prog* P, int i, int64_t r, double* t, int* ht, double* stk, int* near) {
  const int g = P->genes[i];
  const int C = P->C;
  *ht = 0;
  if (g >= SYM_VAR0) return (double)P->X[(int64_t)(g - SYM_VAR0) * P->N + r];
  if (g == SYM_CONST) {
    if (P->duals) {
      memset(t, 0, sizeof(double) * (size_t)C);
      t[P->cidx[i]] = 1.0;
      *ht = 1;
    }
    return P->gc[i];
  }
  const int k = arity(g);
  double* ta = stk;
  double* tb = stk + C;
  double* sub = stk + 2 * C;
  int ha = 0, hb = 0;
  const double a = ev(P, 2 * i + 1, r, ta, &ha, sub, near);
  const double b = k == 2 ? ev(P, 2 * i + 2, r, tb, &hb, sub, near) : 0.0;
  const double G = P->guard, CL = P->clamp;
  double v = 0.0, pa = 0.0, pb = 0.0;
  switch (g) {
    case ADD: v = a + b; pa = 1.0; pb = 1.0; break;
    case SUB: v = a - b; pa = 1.0; pb = -1.0; break;
    case MUL: v = a * b; pa = b; pb = a; break;
    case DIV: {
      const int gd = fabs(b) < G;
      v = gd ? 1.0 : a / b;
      pa = gd ? 0.0 : 1.0 / b;
      pb = gd ? 0.0 : -a / (b * b);
      if (near_thr(b, G, P->window)) *near = 1;
      break;
    }
    case SIN: v = sin(a); pa = cos(a); break;
    case COS: v = cos(a); pa = -sin(a); break;
    case SQ: v = a * a; pa = 2.0 * a; break;
    case SQRT: {
      const double s = sqrt(fabs(a));
      v = s;
      pa = a == 0.0 ? 0.0 : (a > 0.0 ? 1.0 : -1.0) / (2.0 * s);
      break;
    }
    case EXP: {
      v = exp(clampv(a, CL));
      pa = (a >= -CL && a <= CL) ? exp(a) : 0.0;
      if (near_thr(a, CL, P->window)) *near = 1;
      break;
    }
    case LOG: {
      const int gd = fabs(a) < G;
      v = gd ? 0.0 : log(fabs(a));
      pa = gd ? 0.0 : 1.0 / a;
      if (near_thr(a, G, P->window)) *near = 1;
      break;
    }
    case POW: {
      const int gd = fabs(a) < G;
      const double la = gd ? 0.0 : log(fabs(a));
      const double e = b * la;
      v = gd ? 0.0 : exp(clampv(e, CL));
      const int live = !gd && e >= -CL && e <= CL;
      const double rr = live ? exp(e) : 0.0;
      pa = live ? rr * b / a : 0.0;
      pb = live ? rr * la : 0.0;
      if (near_thr(a, G, P->window) || near_thr(gd ? 0.0 : e, CL, P->window)) *near = 1;
      break;
    }
    default: v = NAN; break;
  }
  if (P->duals && (ha || hb)) {
    for (int j = 0; j < C; ++j) {
      double d = 0.0;
      if (ha) d = chain(pa, ta[j]);
      if (hb) d = ha ? d + chain(pb, tb[j]) : chain(pb, tb[j]);
      t[j] = d;
    }
    *ht = 1;
  }
  if (P->eps != 0.0) {
    const double f = 1.0 + P->eps * mca_u(P->seed, i, r);
    v *= f;
    if (*ht)
      for (int j = 0; j < C; ++j) t[j] *= f;
  }
  if (near_thr(v, P->rng_f32 ? F32_MAX : 1.7976931348623157e308, P->window)) *near = 1;
  if (P->rng_f32 && fabs(v) >= F32_OVERFLOW) v = copysign(INFINITY, v);
  return v;
}

typedef struct {
  const Prog* P;
  int64_t r0, r1;
  int pass; /* 0: predictions, 1: gradient terms */
  double* p;
  int nonfinite, near;
  double a, b; /* residual a + b p - y (pass 1) */
  nsum g[MAXC], gabs[MAXC];
} Job;

static void* run_job(void* arg) {
  Job* J = (Job*)arg;
  const Prog* P = J->P;
  const int C = P->C;
  double* buf = (double*)malloc(sizeof(double) * (size_t)C * (2 * MAXDEPTH + 3) + 64);
  double* t = buf;
  double* stk = buf + C;
  for (int64_t r = J->r0; r < J->r1; ++r) {
    int ht = 0, nr = 0;
    const double v = ev(P, 0, r, t, &ht, stk, &nr);
    if (J->pass == 0) {
      J->p[r] = v;
      if (!isfinite(v)) J->nonfinite = 1;
      if (nr) J->near = 1;
    } else if (ht) {
      const double res = J->a + J->b * v - (double)P->y[r];
      for (int j = 0; j < C; ++j) {
        const double term = res * t[j];
        nadd(&J->g[j], term);
        nadd(&J->gabs[j], fabs(term));
      }
    }
  }
  free(buf);
  return NULL;
}

static void run_pass(const Prog* P, int pass, double* p, double a, double b, int nth, Job* jobs) {
  pthread_t th[64];
  if (nth < 1) nth = 1;
  if (nth > 64) nth = 64;
  const int64_t per = (P->N + nth - 1) / nth;
  for (int k = 0; k < nth; ++k) {
    memset(&jobs[k], 0, sizeof(Job));
    jobs[k].P = P;
    jobs[k].r0 = (int64_t)k * per < P->N ? (int64_t)k * per : P->N;
    jobs[k].r1 = jobs[k].r0 + per < P->N ? jobs[k].r0 + per : P->N;
    jobs[k].pass = pass;
    jobs[k].p = p;
    jobs[k].a = a;
    jobs[k].b = b;
    pthread_create(&th[k], NULL, run_job, &jobs[k]);
  }
  for (int k = 0; k < nth; ++k) pthread_join(th[k], NULL);
}

static void post_order_consts(Prog* P, int i, int* n) {
  const int g = P->genes[i];
  const int k = arity(g);
  for (int c = 0; c < k; ++c) post_order_consts(P, 2 * i + 1 + c, n);
  if (g == SYM_CONST) P->cidx[i] = (*n)++;
}

/*
 * Score (and gradient) of one genotype.
 *   genes [T] heap order, gc [T] constants (binary64 holding the binary32
 *   values), X float [F][N] feature-major, y float [N].
 *   thresholds: guard, clamp (the defaults when <= 0), degenerate_rtol.
 *   eps, seed: Monte-Carlo arithmetic (eps = 0: none); window: relative
 *   distance counted as near a decision threshold.
 *   out[0..10): fitness, a, b, mse, nmse, status, near, C, vp (variance of the
 *   predictions), pbar (their mean); then grad[C] and gabs[C] when with_grad.  p_out [N] (may be NULL): the predictions.
 * Returns C (>= 0), or -1 on a malformed genotype / too many constants.
 */
int gg_oracle_run(const int8_t* genes, const double* gc, int T, int height, const float* X, int64_t N,
                  const float* y, int linear_scaling, int rng_f32, double guard, double clamp,
                  double degenerate_rtol, double eps, uint64_t seed, double window, int with_grad,
                  int nthreads, double* out, double* p_out) {
  Prog* P = (Prog*)calloc(1, sizeof(Prog));
  if (!P || T > 1024 || height + 1 > MAXDEPTH) {
    free(P);
    return -1;
  }
  P->genes = genes;
  P->gc = gc;
  P->T = T;
  P->height = height;
  P->X = X;
  P->N = N;
  P->y = y;
  P->rng_f32 = rng_f32;
  P->guard = guard > 0 ? guard : GUARD_DEFAULT;
  P->clamp = clamp > 0 ? clamp : CLAMP_DEFAULT;
  P->window = window;
  P->eps = eps;
  P->seed = seed;
  for (int i = 0; i < T; ++i) P->cidx[i] = -1;
  int nc = 0;
  post_order_consts(P, 0, &nc);
  if (nc > MAXC) {
    free(P);
    return -1;
  }
  P->C = nc;
  P->duals = 0;
  double* p = p_out ? p_out : (double*)malloc(sizeof(double) * (size_t)N);
  Job* jobs = (Job*)calloc(64, sizeof(Job));
  int nth = nthreads;
  if (nth < 1) nth = 1;
  if (nth > 64) nth = 64;
  run_pass(P, 0, p, 0, 0, nth, jobs);
  int nonfinite = 0, near = 0;
  for (int k = 0; k < nth; ++k) {
    nonfinite |= jobs[k].nonfinite;
    near |= jobs[k].near;
  }
  /* target statistics and fit (fitness.score) */
  nsum sy = {0, 0};
  for (int64_t r = 0; r < N; ++r) nadd(&sy, (double)y[r]);
  const double ybar = nval(&sy) / (double)N;
  nsum svy = {0, 0};
  for (int64_t r = 0; r < N; ++r) {
    const double d = (double)y[r] - ybar;
    nadd(&svy, d * d);
  }
  const double vy = nval(&svy) / (double)N;
  double fit, a, b, mse, nmse, vp = NAN, pbar = NAN;
  int status = 0;
  if (nonfinite) {
    status = 1;
    fit = mse = nmse = INFINITY;
    a = ybar;
    b = 0.0;
  } else {
    nsum se = {0, 0}, sp = {0, 0};
    for (int64_t r = 0; r < N; ++r) {
      const double d = p[r] - (double)y[r];
      nadd(&se, d * d);
      nadd(&sp, p[r]);
    }
    mse = nval(&se) / (double)N;
    pbar = nval(&sp) / (double)N;
    nsum spp = {0, 0}, spy = {0, 0};
    for (int64_t r = 0; r < N; ++r) {
      const double dp = p[r] - pbar;
      nadd(&spp, dp * dp);
      nadd(&spy, dp * ((double)y[r] - ybar));
    }
    const double Spp = nval(&spp);
    vp = Spp / (double)N;
    double ls;
    if (vp <= degenerate_rtol * fmax(pbar * pbar, 1e-300)) {
      a = ybar;
      b = 0.0;
      ls = vy;
    } else {
      b = nval(&spy) / Spp;
      a = ybar - b * pbar;
      nsum sr = {0, 0};
      for (int64_t r = 0; r < N; ++r) {
        const double d = (double)y[r] - a - b * p[r];
        nadd(&sr, d * d);
      }
      ls = nval(&sr) / (double)N;
    }
    fit = linear_scaling ? ls : mse;
    nmse = vy > 0 ? fit / vy : (fit == 0.0 ? 0.0 : INFINITY);
  }
  out[0] = fit;
  out[1] = a;
  out[2] = b;
  out[3] = mse;
  out[4] = nmse;
  out[5] = status;
  out[6] = near;
  out[7] = nc;
  out[8] = vp;
  out[9] = pbar;
  if (with_grad) {
    double* g = out + 10;
    double* gabs = out + 10 + nc;
    for (int j = 0; j < nc; ++j) g[j] = gabs[j] = 0.0;
    const int live = status == 0 && nc > 0 && (!linear_scaling || b != 0.0);
    if (live) {
      P->duals = 1;
      const double s0 = linear_scaling ? a : 0.0, s1 = linear_scaling ? b : 1.0;
      run_pass(P, 1, p, s0, s1, nth, jobs);
      const double scale = 2.0 * s1 / (double)N;
      for (int j = 0; j < nc; ++j) {
        nsum tg = {0, 0}, ta = {0, 0};
        for (int k = 0; k < nth; ++k) {
          nadd(&tg, nval(&jobs[k].g[j]));
          nadd(&ta, nval(&jobs[k].gabs[j]));
        }
        g[j] = nval(&tg) * scale;
        gabs[j] = nval(&ta) * fabs(scale);
      }
    }
  }
  free(jobs);
  if (!p_out) free(p);
  free(P);
  return nc;
}
