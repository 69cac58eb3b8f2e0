/*
 * FP64 CPU oracle for the multi-channel VEGAS (VAMP) sample pass.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Plain scalar C,
 * FP64, libm only, built with -ffp-contract=off.  It shares no code with the
 * HIP library.
 *
 * Paper: S. Brass, W. Kilian, J. Reuter, "Parallel Adaptive Monte Carlo
 * Integration with the Event Generator WHIZARD", arXiv:1811.09711.
 * Citations below name the section and the equation label of the paper.
 *
 * Readings where the paper is silent or garbled are marked [Rn]; the list
 * with the reasons sits in the design notes of the repository.
 */
#include "mcv_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define SQRT2 1.41421356237309504880
#define SQRT2PI 2.50662827463100050242
#define INV_SQRTPI 0.56418958354775628695 /* 1/sqrt(pi) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: the counter-based generator of Salmon et al. (SC'11).       */
/* One round multiplies counter words 0 and 2 by the two Philox multipliers,  */
/* and mixes the high halves with words 1, 3 and the key; the key is bumped  */
/* by the two Weyl constants between rounds.  The paper's generators (Sec.    */
/* 4.4) are replaced by this one; what the paper asks of them -- independent, */
/* reproducible streams per worker with no communication -- is kept: every   */
/* word is a pure function of (seed, sample, iteration, word index).          */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    if (r < 9) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
  }
  memcpy(out, c, sizeof c);
}

/* [R2] counter = (i mod 2^32, i / 2^32, t, m / 4), key = (seed mod 2^32, seed / 2^32). */
uint32_t orc_word(uint64_t seed, uint64_t i, uint32_t t, uint32_t m) {
  const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), t, m / 4u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox(ctr, key, out);
  return out[m % 4u];
}

#define TAG_UNWEIGHT 0x80000000u

/* ------------------------------------------------------------------------ */
/* MRG32k3a (Sec. 4.4, eq. mrg32k3a and eq. rngstream; L'Ecuyer's combined  */
/* multiple-recursive generator behind RngStreams).  Two recursions of order */
/* three, x1_n = (1403580 x1_{n-2} - 810728 x1_{n-3}) mod m1 and             */
/* x2_n = (527612 x2_{n-1} - 1370589 x2_{n-3}) mod m2, combined into         */
/* z_n = (x1_n - x2_n) mod m1 (z_n = m1 when that is 0, so u_n = z_n/(m1+1)  */
/* lies in (0,1)).  [Garble: the printed combination modulus 4292967087 is   */
/* m1 = 4294967087.]  A step is a 3x3 matrix on the state vector             */
/* (x_{n-2}, x_{n-1}, x_n); jumps ahead by 2^b steps are powers of it.       */
/* [R28] Streams: the state starts at 12345 in all six words (the RngStreams */
/* package seed); problem seed s and channel c use stream g = 1024 s + c     */
/* (2^127 steps apart), unweighting trials stream 1024 s + 1023; call i of a */
/* channel (its index among the channel's calls) is substream i (2^76 steps  */
/* apart) of its stream, and iteration t starts 64 t steps into it.  Word m  */
/* of a call is floor(z 2^32 / (m1 + 1)) of its (m+1)-th output, so the      */
/* bin / fraction rule [R3] applies unchanged.                              */
/* ------------------------------------------------------------------------ */
#define MRG_M1 4294967087ull
#define MRG_M2 4294944443ull

typedef struct {
  uint64_t a[9]; /* row-major, entries below the modulus */
} mat3;

static mat3 mat3_mul(const mat3* x, const mat3* y, uint64_t mod) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      uint64_t acc = 0;
      for (int k = 0; k < 3; ++k) acc = (acc + (x->a[3 * i + k] * y->a[3 * k + j]) % mod) % mod;
      r.a[3 * i + j] = acc;
    }
  return r;
}

static void mat3_vec(const mat3* x, uint64_t v[3], uint64_t mod) {
  uint64_t r[3];
  for (int i = 0; i < 3; ++i) {
    uint64_t acc = 0;
    for (int k = 0; k < 3; ++k) acc = (acc + (x->a[3 * i + k] * v[k]) % mod) % mod;
    r[i] = acc;
  }
  v[0] = r[0];
  v[1] = r[1];
  v[2] = r[2];
}

/* pow1[b] = A1^(2^b), pow2[b] = A2^(2^b), b = 0..190 (repeated squaring). */
static mat3 mrg_pow1[191], mrg_pow2[191];
static pthread_once_t mrg_once = PTHREAD_ONCE_INIT;

static void mrg_tables(void) {
  const mat3 a1 = {{0, 1, 0, 0, 0, 1, MRG_M1 - 810728u, 1403580u, 0}};
  const mat3 a2 = {{0, 1, 0, 0, 0, 1, MRG_M2 - 1370589u, 0, 527612u}};
  mrg_pow1[0] = a1;
  mrg_pow2[0] = a2;
  for (int b = 1; b < 191; ++b) {
    mrg_pow1[b] = mat3_mul(&mrg_pow1[b - 1], &mrg_pow1[b - 1], MRG_M1);
    mrg_pow2[b] = mat3_mul(&mrg_pow2[b - 1], &mrg_pow2[b - 1], MRG_M2);
  }
}

typedef struct {
  uint64_t x1[3], x2[3];
} mrg_state;

/* The state 2^shift * k steps after st (k < 2^64, shift + 63 <= 190). */
static void mrg_jump(mrg_state* st, int shift, uint64_t k) {
  pthread_once(&mrg_once, mrg_tables);
  for (int b = 0; b < 64 && k; ++b, k >>= 1)
    if (k & 1) {
      mat3_vec(&mrg_pow1[shift + b], st->x1, MRG_M1);
      mat3_vec(&mrg_pow2[shift + b], st->x2, MRG_M2);
    }
}

/* One step: the next z (in [1, m1]). */
static uint32_t mrg_next(mrg_state* st) {
  const uint64_t p1 =
      ((1403580u * st->x1[1]) % MRG_M1 + ((MRG_M1 - 810728u) * st->x1[0]) % MRG_M1) % MRG_M1;
  st->x1[0] = st->x1[1];
  st->x1[1] = st->x1[2];
  st->x1[2] = p1;
  const uint64_t p2 =
      ((527612u * st->x2[2]) % MRG_M2 + ((MRG_M2 - 1370589u) * st->x2[0]) % MRG_M2) % MRG_M2;
  st->x2[0] = st->x2[1];
  st->x2[1] = st->x2[2];
  st->x2[2] = p2;
  const uint64_t z = (p1 + MRG_M1 - p2) % MRG_M1;
  return (uint32_t)(z == 0 ? MRG_M1 : z);
}

/* The start of substream i of stream g, `offset` steps in. */
static mrg_state mrg_start(uint64_t g, uint64_t i, uint64_t offset) {
  mrg_state st = {{12345, 12345, 12345}, {12345, 12345, 12345}};
  mrg_jump(&st, 127, g);
  mrg_jump(&st, 76, i);
  mrg_jump(&st, 0, offset);
  return st;
}

void orc_mrg_outputs(uint64_t g, uint64_t i, uint64_t offset, int32_t count, uint32_t* z) {
  mrg_state st = mrg_start(g, i, offset);
  for (int q = 0; q < count; ++q) z[q] = mrg_next(&st);
}

static uint32_t mrg_word(uint32_t z) {
  return (uint32_t)(((uint64_t)z << 32) / (MRG_M1 + 1));
}

/* Words 0..nw-1 of call i_c of channel c (MRG streams) at iteration t. */
static void mrg_call_words(uint64_t seed, int c, uint64_t i_c, uint32_t t, int nw, uint32_t* u) {
  mrg_state st = mrg_start(1024 * seed + (uint64_t)c, i_c, 64 * (uint64_t)t);
  for (int m = 0; m < nw; ++m) u[m] = mrg_word(mrg_next(&st));
}

/* Words 0..nw-1 of unweighting trial q (MRG streams). */
static void mrg_trial_words(uint64_t seed, uint64_t q, int nw, uint32_t* u) {
  mrg_state st = mrg_start(1024 * seed + 1023, q, 0);
  for (int m = 0; m < nw; ++m) u[m] = mrg_word(mrg_next(&st));
}

/* ------------------------------------------------------------------------ */
/* Inverse complementary error function.  libm has none, so: a starting      */
/* value from the asymptotic form erfc(x) ~ exp(-x^2)/(x sqrt(pi)) (or the   */
/* linear form near x = 0), then Newton steps on erfc(x) - y, which converge */
/* monotonically because erfc is convex and decreasing for x > 0.            */
/* ------------------------------------------------------------------------ */
double orc_erfcinv(double y) {
  if (!(y > 0.0)) return (y == 0.0) ? INFINITY : NAN;
  if (!(y < 2.0)) return (y == 2.0) ? -INFINITY : NAN;
  if (y > 1.0) return -orc_erfcinv(2.0 - y);
  if (y == 1.0) return 0.0;
  double x;
  if (y > 0.5) {
    x = (1.0 - y) * 0.88622692545275801365; /* sqrt(pi)/2 */
  } else {
    x = sqrt(-log(y));
    for (int it = 0; it < 3; ++it) {
      const double v = -log(y * x * 1.77245385090551602730); /* sqrt(pi) */
      if (v > 0.0) x = sqrt(v);
    }
  }
  for (int it = 0; it < 100; ++it) {
    const double d = -2.0 * INV_SQRTPI * exp(-x * x); /* d erfc / dx */
    const double step = (erfc(x) - y) / d;
    x -= step;
    if (fabs(step) <= 1e-17 * fabs(x)) break;
  }
  return x;
}

/* ------------------------------------------------------------------------ */
/* 1-d channel maps (the role of phi_c, Sec. 3.1 and Sec. 3.4).               */
/* Gaussian: truncated normal inverse-CDF on [0,1] [R4].                      */
/* Breit-Wigner: truncated Cauchy inverse-CDF (arctan map), FWHM Gamma [R5]. */
/* Flat: identity.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t kind;
  double loc, width;
  double pa, qb, z;      /* Gauss: Phi(a), 1 - Phi(b), Z = Phi(b) - Phi(a) */
  double h, ta, tb, th;  /* BW: half width, atan bounds, their difference */
} map1d;

static map1d map_setup(int32_t kind, double loc, double width) {
  map1d m;
  memset(&m, 0, sizeof m);
  m.kind = kind;
  m.loc = loc;
  m.width = width;
  if (kind == ORC_GAUSS) {
    const double a = (0.0 - loc) / width, b = (1.0 - loc) / width;
    m.pa = 0.5 * erfc(-a / SQRT2);
    m.qb = 0.5 * erfc(b / SQRT2);
    m.z = (1.0 - m.qb) - m.pa;
  } else if (kind == ORC_BW) {
    m.h = 0.5 * width;
    m.ta = atan((0.0 - loc) / m.h);
    m.tb = atan((1.0 - loc) / m.h);
    m.th = m.tb - m.ta;
  }
  return m;
}

/* x and xc = 1 - x are both passed so the upper tail keeps its precision. */
static double map_forward(const map1d* m, double x, double xc) {
  if (m->kind == ORC_GAUSS) {
    const double t = m->pa + x * m->z;
    double z;
    if (t <= 0.5) {
      z = -SQRT2 * orc_erfcinv(2.0 * t);
    } else {
      const double u = m->qb + xc * m->z; /* = 1 - t */
      z = SQRT2 * orc_erfcinv(2.0 * u);
    }
    return m->loc + m->width * z;
  }
  if (m->kind == ORC_BW) return m->loc + m->h * tan(m->ta + x * m->th);
  return x;
}

static double map_cdf(const map1d* m, double p) {
  if (m->kind == ORC_GAUSS) {
    const double z = (p - m->loc) / m->width;
    if (z <= 0.0) return (0.5 * erfc(-z / SQRT2) - m->pa) / m->z;
    return 1.0 - (0.5 * erfc(z / SQRT2) - m->qb) / m->z;
  }
  if (m->kind == ORC_BW) return (atan((p - m->loc) / m->h) - m->ta) / m->th;
  return p;
}

/* q(p) = 1 / phi'(x): the channel's own density in p (Sec. 3.4). */
static double map_density(const map1d* m, double p) {
  if (m->kind == ORC_GAUSS) {
    const double z = (p - m->loc) / m->width;
    return exp(-0.5 * z * z) / (SQRT2PI * m->width * m->z);
  }
  if (m->kind == ORC_BW) {
    const double u = p - m->loc;
    return m->h / (m->th * (u * u + m->h * m->h));
  }
  return 1.0;
}

/* Untruncated normalised peak factors of the synthetic integrand. */
static double peak_pdf(int32_t kind, double loc, double width, double p) {
  if (kind == ORC_GAUSS) {
    const double z = (p - loc) / width;
    return exp(-0.5 * z * z) / (SQRT2PI * width);
  }
  if (kind == ORC_BW) {
    const double h = 0.5 * width, u = p - loc;
    return h / (M_PI * (u * u + h * h));
  }
  return 1.0;
}

double orc_map_forward(int32_t kind, double loc, double width, double x) {
  map1d m = map_setup(kind, loc, width);
  return map_forward(&m, x, 1.0 - x);
}
double orc_map_cdf(int32_t kind, double loc, double width, double p) {
  map1d m = map_setup(kind, loc, width);
  return map_cdf(&m, p);
}
double orc_map_density(int32_t kind, double loc, double width, double p) {
  map1d m = map_setup(kind, loc, width);
  return map_density(&m, p);
}
double orc_peak_pdf(int32_t kind, double loc, double width, double p) {
  return peak_pdf(kind, loc, width, p);
}

/* ------------------------------------------------------------------------ */
/* State                                                                      */
/* ------------------------------------------------------------------------ */
struct orc_state {
  int32_t d, K, n, P, fp32, rng, strat;
  uint64_t seed;
  double grid_power, channel_power;
  int64_t min_calls;
  int32_t* pk;
  double *pl, *pw, *pwt;
  map1d* maps;     /* [K][d] */
  double* edges;   /* [K][d][n+1] */
  double* alpha;   /* [K] */
  int64_t* nc;     /* [K] */
  int64_t* start;  /* [K+1] */
  int64_t *nr, *spb; /* [K] stratified mode: boxes per axis, calls per box */
  double* ssw_c;     /* [K] stratified mode: sum over boxes of the squared deviations of
                      * the box's weights from the box mean */
  int64_t ntot;
  int64_t iteration;
  /* last pass, per channel */
  double *s1, *s2, *wmax_c, *e_c, *w_c, *v_c;
  int64_t* nbad_c;
  double* hist;    /* [K][d][n] */
  int32_t max_iter, n_iter;
  double* history; /* [max_iter][5] */
  double wmax_unw;
  int64_t trials_done;
  int64_t last_n;      /* n_points of the last allocation */
  int32_t alloc_valid; /* alpha still equals N_c / N_tot of that allocation */
  int32_t n_eq;        /* channel equivalences: [n_eq][2 + 2d] = c, c', perm[d], mode[d] */
  int32_t* eq;
};

#define EDGE(s, c, k) ((s)->edges + ((size_t)(c) * (s)->d + (k)) * ((s)->n + 1))
#define HIST(s, c, k) ((s)->hist + ((size_t)(c) * (s)->d + (k)) * (s)->n)

/* [R14] precision mode: edges rounded to FP32, then kept strictly increasing
 * in FP32 (forward, then backward pass). */
static void snap_axis32(int32_t n, double* e) {
  float f[257];
  for (int i = 0; i <= n; ++i) f[i] = (float)e[i];
  f[0] = 0.0f;
  f[n] = 1.0f;
  for (int i = 1; i < n; ++i)
    if (!(f[i] > f[i - 1])) f[i] = nextafterf(f[i - 1], 2.0f);
  for (int i = n - 1; i >= 1; --i)
    if (!(f[i] < f[i + 1])) f[i] = nextafterf(f[i + 1], -1.0f);
  for (int i = 0; i <= n; ++i) e[i] = (double)f[i];
}

orc_state* orc_create(const orc_problem* pr, int32_t max_iter) {
  if (!pr || pr->dim < 1 || pr->dim > 32 || pr->n_bins < 1 || pr->n_bins > 256 ||
      pr->n_channels < 1 || pr->n_peaks < 1 || max_iter < 1)
    return NULL;
  if (pr->rng != 0 && (pr->rng != 1 || pr->n_channels > 1023 || pr->seed >= ((uint64_t)1 << 54)))
    return NULL;
  orc_state* s = (orc_state*)calloc(1, sizeof *s);
  const int32_t d = pr->dim, K = pr->n_channels, n = pr->n_bins, P = pr->n_peaks;
  s->d = d;
  s->K = K;
  s->n = n;
  s->P = P;
  s->fp32 = pr->fp32_rules ? 1 : 0;
  s->rng = pr->rng;
  if (pr->strat == 1 || pr->strat < 0) {
    free(s);
    return NULL;
  }
  s->strat = pr->strat;
  s->seed = pr->seed;
  s->grid_power = pr->grid_power;
  s->channel_power = pr->channel_power;
  s->min_calls = pr->min_calls;
  s->pk = (int32_t*)malloc(sizeof(int32_t) * P * d);
  s->pl = (double*)malloc(sizeof(double) * P * d);
  s->pw = (double*)malloc(sizeof(double) * P * d);
  s->pwt = (double*)malloc(sizeof(double) * P);
  memcpy(s->pk, pr->peak_kind, sizeof(int32_t) * P * d);
  memcpy(s->pl, pr->peak_loc, sizeof(double) * P * d);
  memcpy(s->pw, pr->peak_width, sizeof(double) * P * d);
  memcpy(s->pwt, pr->peak_weight, sizeof(double) * P);
  s->maps = (map1d*)malloc(sizeof(map1d) * K * d);
  for (int c = 0; c < K; ++c)
    for (int k = 0; k < d; ++k)
      s->maps[c * d + k] = map_setup(pr->chan_kind[c * d + k], pr->chan_loc[c * d + k],
                                     pr->chan_width[c * d + k]);
  /* Initial grids: equidistant bins (Sec. 3.2 and Sec. 3.5); alpha_c = 1/K
   * (Sec. 3.4). */
  s->edges = (double*)malloc(sizeof(double) * K * d * (n + 1));
  for (int c = 0; c < K; ++c)
    for (int k = 0; k < d; ++k) {
      double* e = EDGE(s, c, k);
      for (int j = 0; j <= n; ++j) e[j] = (double)j / (double)n;
      if (s->fp32) snap_axis32(n, e);
    }
  s->alpha = (double*)malloc(sizeof(double) * K);
  for (int c = 0; c < K; ++c) s->alpha[c] = 1.0 / (double)K;
  s->nc = (int64_t*)calloc(K, sizeof(int64_t));
  s->start = (int64_t*)calloc(K + 1, sizeof(int64_t));
  s->nr = (int64_t*)calloc(K, sizeof(int64_t));
  s->spb = (int64_t*)calloc(K, sizeof(int64_t));
  s->ssw_c = (double*)calloc(K, sizeof(double));
  s->s1 = (double*)calloc(K, sizeof(double));
  s->s2 = (double*)calloc(K, sizeof(double));
  s->wmax_c = (double*)calloc(K, sizeof(double));
  s->e_c = (double*)calloc(K, sizeof(double));
  s->w_c = (double*)calloc(K, sizeof(double));
  s->v_c = (double*)calloc(K, sizeof(double));
  s->nbad_c = (int64_t*)calloc(K, sizeof(int64_t));
  s->hist = (double*)calloc((size_t)K * d * n, sizeof(double));
  s->max_iter = max_iter;
  s->history = (double*)calloc((size_t)max_iter * 5, sizeof(double));
  s->wmax_unw = -1.0;
  return s;
}

void orc_destroy(orc_state* s) {
  if (!s) return;
  free(s->pk); free(s->pl); free(s->pw); free(s->pwt); free(s->maps);
  free(s->edges); free(s->alpha); free(s->nc); free(s->start);
  free(s->nr); free(s->spb); free(s->ssw_c);
  free(s->s1); free(s->s2); free(s->wmax_c); free(s->e_c); free(s->w_c);
  free(s->v_c); free(s->nbad_c); free(s->hist); free(s->history); free(s->eq);
  free(s);
}

/* ------------------------------------------------------------------------ */
/* Channel allocation (Sec. 3.4, after eq. 15): N_c = alpha_c N made integer; */
/* channels that would get very few calls are held at a floor N_min ("say    */
/* N_c = 10"); N may be adjusted so that all N_c are integers.  [R16] floor,  */
/* never switch off.  Remainder by largest fractional part, ties to lower c. */
/* ------------------------------------------------------------------------ */
int orc_allocation(int32_t K, const double* alpha, int64_t n_points, int64_t min_calls,
                   int64_t* nc, double* alpha_out) {
  double* frac = (double*)malloc(sizeof(double) * K);
  int8_t* taken = (int8_t*)calloc(K, 1);
  int64_t sum = 0;
  for (int c = 0; c < K; ++c) {
    const double v = alpha[c] * (double)n_points;
    const double fl = floor(v);
    int64_t b = (int64_t)fl;
    frac[c] = v - fl;
    if (b < min_calls) {
      b = min_calls;
      frac[c] = -1.0;
    }
    nc[c] = b;
    sum += b;
  }
  int64_t rem = n_points - sum;
  while (rem > 0) {
    int best = -1;
    for (int c = 0; c < K; ++c)
      if (!taken[c] && (best < 0 || frac[c] > frac[best])) best = c;
    if (best < 0) {
      memset(taken, 0, K);
      continue;
    }
    nc[best] += 1;
    taken[best] = 1;
    --rem;
  }
  int64_t ntot = 0;
  for (int c = 0; c < K; ++c) ntot += nc[c];
  for (int c = 0; c < K; ++c) alpha_out[c] = (double)nc[c] / (double)ntot;
  free(frac);
  free(taken);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* (Pseudo-)stratified sampling (Sec. 3.3): r space of a channel is cut into */
/* nr^d equal boxes and every box gets the same number of calls, at least s  */
/* (s >= 2), each uniform inside its box; the VEGAS map then carries r to x  */
/* (pseudo-stratification: the boxes are not the grid's bins).  [R30] A      */
/* channel's N_c calls from the allocation give nr = the largest integer     */
/* with s nr^d <= N_c (at most 2^20), calls per box floor(N_c / nr^d), and   */
/* the channel then takes calls per box times nr^d calls (the paper fixes N  */
/* = s n^d; Sec. 3.4 lets N and alpha be adjusted to whole numbers of calls). */
/* ------------------------------------------------------------------------ */
void orc_strat_layout(int64_t n, int32_t d, int64_t s_min, int64_t* nr, int64_t* per_box) {
  int64_t r = 1;
  for (;;) {
    const int64_t r1 = r + 1;
    if (r1 > ((int64_t)1 << 20)) break;
    int64_t boxes = 1;
    int over = 0;
    for (int k = 0; k < d && !over; ++k) {
      if (boxes > n / r1) over = 1;
      else boxes *= r1;
    }
    if (over || boxes > n / s_min) break;
    r = r1;
  }
  int64_t boxes = 1;
  for (int k = 0; k < d; ++k) boxes *= r;
  *nr = r;
  *per_box = n / boxes;
}

/* Rounds each N_c of an allocation to whole boxes (stratified mode) and
 * re-derives N_tot and alpha = N_c / N_tot. */
static void strat_adjust(int32_t K, int32_t d, int64_t s_min, int64_t* nc, int64_t* nr,
                         int64_t* spb, double* alpha_out) {
  int64_t tot = 0;
  for (int c = 0; c < K; ++c) {
    orc_strat_layout(nc[c], d, s_min, &nr[c], &spb[c]);
    int64_t boxes = 1;
    for (int k = 0; k < d; ++k) boxes *= nr[c];
    nc[c] = spb[c] * boxes;
    tot += nc[c];
  }
  for (int c = 0; c < K; ++c) alpha_out[c] = (double)nc[c] / (double)tot;
}

int orc_allocate(orc_state* s, int64_t n_points) {
  if (n_points < 1) return -1;
  orc_allocation(s->K, s->alpha, n_points, s->min_calls, s->nc, s->alpha);
  if (s->strat) strat_adjust(s->K, s->d, s->strat, s->nc, s->nr, s->spb, s->alpha);
  s->start[0] = 0;
  for (int c = 0; c < s->K; ++c) s->start[c + 1] = s->start[c] + s->nc[c];
  s->ntot = s->start[s->K];
  s->last_n = n_points;
  s->alloc_valid = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One point (Sec. 3.5, the paragraph organising an iteration; eq. g(p)).    */
/* ------------------------------------------------------------------------ */
typedef struct {
  double f, g, w;
} point_result;

/* Largest j in [0, n-1] with e[j] <= x (Sec. 3.2: x lies in bin B_j). */
static int find_bin(const double* e, int n, double x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (e[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

/* [R3] bin j = floor(u n / 2^32) and the remaining fraction of u n. */
static void bin_frac(uint32_t u, int n, int fp32, int* j, double* frac) {
  const uint64_t prod = (uint64_t)u * (uint64_t)n;
  const uint32_t lo = (uint32_t)prod;
  *j = (int)(prod >> 32);
  if (fp32) *frac = ((double)(lo >> 9) + 0.5) * 0x1p-23;
  else *frac = ((double)lo + 0.5) * 0x1p-32;
}

/* The integrand f(p) = sum_i w_i prod_k pdf_ik(p_k). */
static double integrand(const orc_state* s, const double* p) {
  double f = 0.0;
  for (int i = 0; i < s->P; ++i) {
    double v = s->pwt[i];
    for (int k = 0; k < s->d; ++k)
      v *= peak_pdf(s->pk[i * s->d + k], s->pl[i * s->d + k], s->pw[i * s->d + k], p[k]);
    f += v;
  }
  return f;
}

/* Evaluate the point with words u[0..d-1] in channel c.  Sec. 3.2 eq. g(x)
 * for the own grid density, Sec. 3.5 eq. g(p) for the multi-channel density
 * (read with x_c = phi_c^{-1}(p) [R8]), w = f/g (eq. vamp-master).
 * Optional outputs: own bins, all-channel bins [K][d], near-edge flags, p. */
/* [R30] stratified mode: r = (b + u 2^-32) / nr for box digit b, as the
 * fixed-point R = b 2^32 + u over nr 2^32; j = floor(R n / (nr 2^32)), rem =
 * R n - j nr 2^32, fraction (rem + 1/2) / (nr 2^32) (one correctly rounded
 * division; exact for nr a power of two); FP32 rules round it to FP32 (the
 * largest float below 1 if that rounds to 1).  nr = 1 gives [R3]'s bin. */
static void strat_bin_frac(uint32_t u, int64_t b, int64_t nr, int n, int fp32, int* j,
                           double* frac) {
  const unsigned __int128 R = ((unsigned __int128)b << 32) | u;
  const unsigned __int128 Rn = R * (unsigned __int128)n;
  const unsigned __int128 D = (unsigned __int128)nr << 32;
  *j = (int)(Rn / D);
  const uint64_t rem = (uint64_t)(Rn - (unsigned __int128)(*j) * D);
  double f = ((double)rem + 0.5) / ((double)nr * 4294967296.0);
  if (fp32) {
    float g = (float)f;
    if (g >= 1.0f) g = nextafterf(1.0f, 0.0f);
    f = (double)g;
  }
  *frac = f;
}

/* (bin, fraction) of every axis of call i_c of channel c from its words:
 * [R3], or [R30] with the call's box when nr / spb are given. */
static void call_bins(const orc_state* s, const int64_t* nr, const int64_t* spb, int c,
                      int64_t i_c, const uint32_t* u, int* jb, double* fr) {
  if (!s->strat) {
    for (int k = 0; k < s->d; ++k) bin_frac(u[k], s->n, s->fp32, &jb[k], &fr[k]);
    return;
  }
  int64_t q = i_c / spb[c]; /* the call's box; digit k of q in base nr is its axis-k stratum */
  for (int k = 0; k < s->d; ++k) {
    const int64_t b = q % nr[c];
    q /= nr[c];
    strat_bin_frac(u[k], b, nr[c], s->n, s->fp32, &jb[k], &fr[k]);
  }
}

static point_result eval_point(const orc_state* s, int c, const int* jin, const double* fin,
                               int* own_bins, int32_t* all_bins, uint8_t* near, double* p_out) {
  const int d = s->d, n = s->n, K = s->K;
  double p[32];
  int jb[32];
  double own_g = 1.0;
  for (int k = 0; k < d; ++k) {
    const double frac = fin[k];
    jb[k] = jin[k];
    const double* e = EDGE(s, c, k);
    const double w = e[jb[k] + 1] - e[jb[k]];
    const double x = e[jb[k]] + frac * w;
    const double xc = (1.0 - e[jb[k] + 1]) + (1.0 - frac) * w;
    p[k] = map_forward(&s->maps[c * d + k], x, xc);
    own_g *= 1.0 / ((double)n * w);
  }
  const double f = integrand(s, p);
  double g = 0.0;
  for (int cc = 0; cc < K; ++cc) {
    double q = 1.0, gc = 1.0;
    for (int k = 0; k < d; ++k) {
      const map1d* m = &s->maps[cc * d + k];
      q *= map_density(m, p[k]);
      if (cc != c) {
        const double xp = map_cdf(m, p[k]);
        const double* e = EDGE(s, cc, k);
        const int J = find_bin(e, n, xp);
        gc *= 1.0 / ((double)n * (e[J + 1] - e[J]));
        if (all_bins) all_bins[cc * d + k] = J;
        if (near) {
          uint8_t fl = 0;
          if (J >= 1 && fabs(xp - e[J]) < 1e-12) fl = 1;
          if (J + 1 <= n - 1 && fabs(xp - e[J + 1]) < 1e-12) fl = 1;
          near[cc * d + k] = fl;
        }
      } else {
        if (all_bins) all_bins[cc * d + k] = jb[k];
        if (near) near[cc * d + k] = 0;
      }
    }
    if (cc == c) gc = own_g;
    g += s->alpha[cc] * gc * q;
  }
  if (own_bins)
    for (int k = 0; k < d; ++k) own_bins[k] = jb[k];
  if (p_out)
    for (int k = 0; k < d; ++k) p_out[k] = p[k];
  point_result r = {f, g, f / g};
  return r;
}

static int channel_of(const int64_t* start, int K, int64_t i) {
  int c = 0;
  while (c < K - 1 && i >= start[c + 1]) ++c;
  return c;
}

/* Neumaier's compensated summation. */
static void neumaier(double* sum, double* comp, double v) {
  const double t = *sum + v;
  if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
  else *comp += (v - t) + *sum;
  *sum = t;
}

typedef struct {
  const orc_state* s;
  int64_t lo, hi;
  uint32_t tag;
  double *s1, *c1, *s2, *c2, *wmax;
  int64_t* nbad;
  double* hist;
  double *ssw, *cssw; /* stratified mode: per channel, the (compensated) sum over
                       * boxes of the squared deviations from the box mean */
} pass_job;

/* Sum of the squared deviations of k weights from their mean, in two passes
 * (the mean first, then the deviations), so that no digits cancel however
 * little the weights spread. */
static double box_ssw(const double* w, int64_t k) {
  if (k < 2) return 0.0;
  double sum = 0.0, comp = 0.0;
  for (int64_t i = 0; i < k; ++i) neumaier(&sum, &comp, w[i]);
  const double mean = (sum + comp) / (double)k;
  double ss = 0.0, cs = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    const double e = w[i] - mean;
    neumaier(&ss, &cs, e * e);
  }
  return ss + cs;
}

/* Sample points [lo, hi): Sec. 3.2 eq. 4 (sums of w and w^2), eq. 31 (per-bin
 * sums of w^2 along each axis, own channel only [R9a]). */
static void* pass_worker(void* arg) {
  pass_job* jb = (pass_job*)arg;
  const orc_state* s = jb->s;
  const int d = s->d, n = s->n, K = s->K;
  const int nw = d;
  uint32_t u[32];
  int bins[32], jin[32];
  double fin[32];
  /* stratified mode: the finite weights of the current box */
  int box_c = -1;
  int64_t box_q = -1, box_k = 0;
  double* boxw = NULL;
  if (s->strat) {
    int64_t mmax = 1;
    for (int c = 0; c < K; ++c)
      if (s->spb[c] > mmax) mmax = s->spb[c];
    boxw = (double*)malloc((size_t)mmax * sizeof(double));
  }
  for (int64_t i = jb->lo; i < jb->hi; ++i) {
    const int c = channel_of(s->start, K, i);
    const int64_t i_c = i - s->start[c];
    if (s->strat) { /* a new box: its spread goes to the channel's variance */
      const int64_t q = i_c / s->spb[c];
      if (c != box_c || q != box_q) {
        if (box_c >= 0) neumaier(&jb->ssw[box_c], &jb->cssw[box_c], box_ssw(boxw, box_k));
        box_c = c;
        box_q = q;
        box_k = 0;
      }
    }
    if (s->rng)
      mrg_call_words(s->seed, c, (uint64_t)i_c, jb->tag, nw, u);
    else
      for (int m = 0; m < nw; ++m) u[m] = orc_word(s->seed, (uint64_t)i, jb->tag, (uint32_t)m);
    call_bins(s, s->nr, s->spb, c, i_c, u, jin, fin);
    const point_result r = eval_point(s, c, jin, fin, bins, NULL, NULL, NULL);
    const double w = r.w;
    if (!isfinite(w)) { /* [R7] counted and excluded */
      jb->nbad[c] += 1;
      continue;
    }
    if (s->strat) boxw[box_k++] = w;
    neumaier(&jb->s1[c], &jb->c1[c], w);
    neumaier(&jb->s2[c], &jb->c2[c], w * w);
    if (fabs(w) > jb->wmax[c]) jb->wmax[c] = fabs(w); /* [R27] largest |w| */
    for (int k = 0; k < d; ++k) jb->hist[((size_t)c * d + k) * n + bins[k]] += w * w;
  }
  if (box_c >= 0) neumaier(&jb->ssw[box_c], &jb->cssw[box_c], box_ssw(boxw, box_k));
  free(boxw);
  return NULL;
}

/* First call of the worker ranges: thread t of T starts at N t / T, moved
 * back to the start of its box in stratified mode (boxes are whole within a
 * channel and channels start on a box), so that no box is split. */
static int64_t worker_start(const orc_state* s, int t, int T) {
  int64_t lo = s->ntot * t / T;
  if (s->strat && lo < s->ntot) {
    const int c = channel_of(s->start, s->K, lo);
    lo = s->start[c] + (lo - s->start[c]) / s->spb[c] * s->spb[c];
  }
  return lo;
}

int orc_sample_iteration(orc_state* s, int64_t n_points, int32_t n_threads) {
  if (s->n_iter >= s->max_iter) return -4;
  if (n_points < (int64_t)s->K * s->min_calls) return -1;
  if (n_threads < 1) n_threads = 1;
  orc_allocate(s, n_points);
  const int K = s->K, d = s->d, n = s->n;
  const size_t hsz = (size_t)K * d * n;
  pass_job* jobs = (pass_job*)calloc(n_threads, sizeof(pass_job));
  pthread_t* th = (pthread_t*)calloc(n_threads, sizeof(pthread_t));
  for (int t = 0; t < n_threads; ++t) {
    pass_job* jb = &jobs[t];
    jb->s = s;
    jb->lo = worker_start(s, t, n_threads);
    jb->hi = t + 1 < n_threads ? worker_start(s, t + 1, n_threads) : s->ntot;
    jb->tag = (uint32_t)s->iteration;
    jb->s1 = (double*)calloc(K, sizeof(double));
    jb->c1 = (double*)calloc(K, sizeof(double));
    jb->s2 = (double*)calloc(K, sizeof(double));
    jb->c2 = (double*)calloc(K, sizeof(double));
    jb->wmax = (double*)calloc(K, sizeof(double));
    jb->nbad = (int64_t*)calloc(K, sizeof(int64_t));
    jb->hist = (double*)calloc(hsz, sizeof(double));
    jb->ssw = (double*)calloc(K, sizeof(double));
    jb->cssw = (double*)calloc(K, sizeof(double));
    if (n_threads > 1) pthread_create(&th[t], NULL, pass_worker, jb);
  }
  if (n_threads == 1) pass_worker(&jobs[0]);
  else
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);

  /* Combine the workers in order, then finalize per channel (Sec. 3.1 E_N,
   * V_N; Sec. 3.4 multi-channel estimator). */
  memset(s->hist, 0, hsz * sizeof(double));
  double e_tot = 0.0, var = 0.0, wmax = 0.0;
  int64_t nbad = 0;
  for (int c = 0; c < K; ++c) {
    double a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0, a3 = 0.0, b3 = 0.0, wm = 0.0;
    int64_t nb = 0;
    for (int t = 0; t < n_threads; ++t) {
      neumaier(&a1, &b1, jobs[t].s1[c]);
      neumaier(&a1, &b1, jobs[t].c1[c]);
      neumaier(&a2, &b2, jobs[t].s2[c]);
      neumaier(&a2, &b2, jobs[t].c2[c]);
      if (jobs[t].wmax[c] > wm) wm = jobs[t].wmax[c];
      nb += jobs[t].nbad[c];
      neumaier(&a3, &b3, jobs[t].ssw[c]);
      neumaier(&a3, &b3, jobs[t].cssw[c]);
    }
    s->ssw_c[c] = a3 + b3;
    s->s1[c] = a1 + b1;
    s->s2[c] = a2 + b2;
    s->wmax_c[c] = wm;
    s->nbad_c[c] = nb;
    const double N = (double)s->nc[c];
    s->e_c[c] = s->s1[c] / N;
    s->w_c[c] = s->s2[c] / N;
    if (s->strat) {
      /* [R30] stratified sampling: the variance of the channel's sum is the
       * sum over its boxes of m sigma_b^2 (m calls per box), estimated in
       * each box by the sample variance of its weights, SSW_b / (m - 1) with
       * SSW_b the squared deviations from the box mean:
       * Var(S1) = m/(m-1) sum_b SSW_b (the same as m/(m-1) (S2 - Q/m), Q the
       * sum of squared box sums, without the cancellation of that form);
       * V_c is that divided by N_c, so that Var(E_c) = V_c / N_c as below. */
      const double m = (double)s->spb[c];
      const double v = (m / (m - 1.0)) * s->ssw_c[c] / N;
      s->v_c[c] = v > 0.0 ? v : 0.0;
    } else {
      const double v = s->w_c[c] - s->e_c[c] * s->e_c[c];
      s->v_c[c] = (s->nc[c] > 1) ? (v > 0.0 ? v : 0.0) * N / (N - 1.0) : 0.0;
    }
    e_tot += s->s1[c];
    const double frac = N / (double)s->ntot;
    var += frac * frac * s->v_c[c] / N;
    if (wm > wmax) wmax = wm;
    nbad += nb;
  }
  for (int t = 0; t < n_threads; ++t)
    for (size_t h = 0; h < hsz; ++h) s->hist[h] += jobs[t].hist[h];
  e_tot /= (double)s->ntot;
  /* [R10] the error is sqrt(V/N), consistent with eq. error-scaling. */
  double* rec = s->history + (size_t)s->n_iter * 5;
  rec[0] = e_tot;
  rec[1] = sqrt(var);
  rec[2] = (double)s->ntot;
  rec[3] = wmax;
  rec[4] = (double)nbad;
  s->n_iter += 1;
  s->iteration += 1;
  for (int t = 0; t < n_threads; ++t) {
    free(jobs[t].s1); free(jobs[t].c1); free(jobs[t].s2); free(jobs[t].c2);
    free(jobs[t].wmax); free(jobs[t].nbad); free(jobs[t].hist); free(jobs[t].ssw);
    free(jobs[t].cssw);
  }
  free(jobs);
  free(th);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Grid refinement, one axis (Sec. 3.2, eq. 30 and eq. 31).                   */
/* omega_j = sqrt(sum of w^2 in bin j); r_j = omega_j / sum omega;            */
/* m_j = ((r_j - 1)/ln r_j)^power, with the limits m = 0 at r = 0 and m = 1  */
/* at r = 1.  New edges split the total measure M = sum m_j into n equal     */
/* parts, taking m as uniform inside each old bin [R11, R12, R13].            */
/* ------------------------------------------------------------------------ */
int orc_rebin_axis(int32_t n, const double* e, const double* h, double power, int32_t snap32,
                   double* out) {
  double omega[256], m[256];
  double sum = 0.0;
  for (int j = 0; j < n; ++j) {
    omega[j] = sqrt(h[j]);
    sum += omega[j];
  }
  if (!(sum > 0.0) || !isfinite(sum)) {
    for (int j = 0; j <= n; ++j) out[j] = e[j];
    if (snap32) snap_axis32(n, out);
    return 0;
  }
  double M = 0.0;
  for (int j = 0; j < n; ++j) {
    const double r = omega[j] / sum;
    if (r == 0.0) m[j] = 0.0;
    else if (r == 1.0) m[j] = 1.0;
    else m[j] = pow((r - 1.0) / log(r), power);
    M += m[j];
  }
  out[0] = 0.0;
  double acc = 0.0;
  int j = 0;
  for (int i = 1; i < n; ++i) {
    const double target = ((double)i * M) / (double)n;
    while (j < n - 1 && (m[j] == 0.0 || acc + m[j] < target)) {
      acc += m[j];
      ++j;
    }
    out[i] = e[j] + ((target - acc) / m[j]) * (e[j + 1] - e[j]);
  }
  out[n] = 1.0;
  for (int i = 1; i < n; ++i)
    if (!(out[i] > out[i - 1])) out[i] = nextafter(out[i - 1], 2.0);
  for (int i = n - 1; i >= 1; --i)
    if (!(out[i] < out[i + 1])) out[i] = nextafter(out[i + 1], -1.0);
  if (snap32) snap_axis32(n, out);
  return 0;
}

/* Channel-weight update, eq. 15: alpha_c <- alpha_c w_c^beta / sum.  [R9]
 * omega_c is the channel's second moment of the weights W_c = S2_c / N_c. */
int orc_update_alpha(int32_t K, double* alpha, const double* w2, double beta) {
  double den = 0.0;
  for (int c = 0; c < K; ++c) den += alpha[c] * pow(w2[c], beta);
  if (!(den > 0.0) || !isfinite(den)) return 0;
  for (int c = 0; c < K; ++c) alpha[c] = alpha[c] * pow(w2[c], beta) / den;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Channel equivalences (Sec. 3.5, the similarity mappings between channels  */
/* that share a structure).  An equivalence (c, c', pi, mode) adds channel    */
/* c''s bin weights along axis pi(k) to the weights channel c is rebinned     */
/* with along axis k; per axis the mode is                                    */
/*   identity:  w_j += w'_j                                                   */
/*   invert:    w_j += w'_{n-1-j}            [R26: the printed d - j read as  */
/*                                            the mirrored bin]              */
/*   symmetric: w_j += (w'_j + w'_{n-1-j}) / 2                                */
/*   invariant: w_j = 1 (the axis keeps its grid)                             */
/* [R26] the bin weights are the per-bin sums of w^2 of eq. 31 of the pass.  */
/* A channel named on the left of any equivalence is rebinned with the sum   */
/* of its equivalences only, added in list order from zero: its own weights  */
/* enter through the trivial equivalence (c, c, identity), which a list      */
/* names explicitly.  Channels named on no left side keep their own weights. */
/* ------------------------------------------------------------------------ */
enum { EQ_IDENTITY = 0, EQ_INVERT = 1, EQ_SYMMETRIC = 2, EQ_INVARIANT = 3 };

int orc_set_equivalences(orc_state* s, int32_t n_eq, const int32_t* eq) {
  const int d = s->d, rec = 2 + 2 * d;
  if (n_eq < 0 || (n_eq > 0 && !eq)) return -1;
  for (int e = 0; e < n_eq; ++e) {
    const int32_t* r = eq + (size_t)e * rec;
    if (r[0] < 0 || r[0] >= s->K || r[1] < 0 || r[1] >= s->K) return -1;
    int seen[32] = {0};
    for (int k = 0; k < d; ++k) {
      if (r[2 + k] < 0 || r[2 + k] >= d || seen[r[2 + k]]++) return -1; /* a permutation */
      if (r[2 + d + k] < EQ_IDENTITY || r[2 + d + k] > EQ_INVARIANT) return -1;
    }
  }
  free(s->eq);
  s->eq = NULL;
  s->n_eq = n_eq;
  if (n_eq > 0) {
    s->eq = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_eq * rec);
    memcpy(s->eq, eq, sizeof(int32_t) * (size_t)n_eq * rec);
  }
  return 0;
}

/* The bin weights of channel c, axis k after the equivalences -> out[n]. */
static void equivalent_weights(const orc_state* s, int c, int k, double* out) {
  const int d = s->d, n = s->n, rec = 2 + 2 * d;
  const double* h = HIST(s, c, k);
  int invariant = 0, listed = 0;
  for (int e = 0; e < s->n_eq; ++e) listed |= s->eq[(size_t)e * rec] == c;
  for (int j = 0; j < n; ++j) out[j] = listed ? 0.0 : h[j];
  for (int e = 0; e < s->n_eq; ++e) {
    const int32_t* r = s->eq + (size_t)e * rec;
    if (r[0] != c) continue;
    const double* h2 = HIST(s, r[1], r[2 + k]);
    switch (r[2 + d + k]) {
      case EQ_IDENTITY:
        for (int j = 0; j < n; ++j) out[j] += h2[j];
        break;
      case EQ_INVERT:
        for (int j = 0; j < n; ++j) out[j] += h2[n - 1 - j];
        break;
      case EQ_SYMMETRIC:
        for (int j = 0; j < n; ++j) out[j] += 0.5 * (h2[j] + h2[n - 1 - j]);
        break;
      default:
        invariant = 1;
    }
  }
  if (invariant)
    for (int j = 0; j < n; ++j) out[j] = 1.0;
}

int orc_get_equivalent_hist(const orc_state* s, double* out) {
  for (int c = 0; c < s->K; ++c)
    for (int k = 0; k < s->d; ++k)
      equivalent_weights(s, c, k, out + ((size_t)c * s->d + k) * s->n);
  return 0;
}

int orc_refine(orc_state* s, uint32_t what) {
  if (s->n_iter == 0) return -4;
  if (what & ORC_REFINE_GRID) {
    const size_t hsz = (size_t)s->K * s->d * s->n;
    double* w = (double*)malloc(sizeof(double) * hsz);
    orc_get_equivalent_hist(s, w);
    double out[257];
    for (int c = 0; c < s->K; ++c)
      for (int k = 0; k < s->d; ++k) {
        orc_rebin_axis(s->n, EDGE(s, c, k), w + ((size_t)c * s->d + k) * s->n, s->grid_power,
                       s->fp32, out);
        memcpy(EDGE(s, c, k), out, sizeof(double) * (s->n + 1));
      }
    free(w);
  }
  if (what & ORC_REFINE_ALPHA) {
    orc_update_alpha(s->K, s->alpha, s->w_c, s->channel_power);
    s->alloc_valid = 0;
  }
  return 0;
}

/* Combination of iterations (Sec. 3.5, last paragraph of the iteration
 * organisation) [R17]: inverse-variance weighted mean, its error, chi^2/ndf. */
int orc_result(const orc_state* s, int32_t first, double out[4]) {
  if (s->n_iter == 0 || first < 0 || first >= s->n_iter) return -4;
  double sw = 0.0, swe = 0.0, zsum = 0.0;
  int nz = 0, nused = 0;
  for (int t = first; t < s->n_iter; ++t) {
    const double e = s->history[t * 5 + 0], sg = s->history[t * 5 + 1];
    ++nused;
    if (sg == 0.0) {
      zsum += e;
      ++nz;
    } else {
      sw += 1.0 / (sg * sg);
      swe += e / (sg * sg);
    }
  }
  if (nz > 0) {
    out[0] = zsum / nz;
    out[1] = 0.0;
    out[2] = 0.0;
    out[3] = nused;
    return 0;
  }
  const double mean = swe / sw;
  double chi2 = 0.0;
  for (int t = first; t < s->n_iter; ++t) {
    const double e = s->history[t * 5 + 0], sg = s->history[t * 5 + 1];
    chi2 += (e - mean) * (e - mean) / (sg * sg);
  }
  out[0] = mean;
  out[1] = 1.0 / sqrt(sw);
  out[2] = (nused > 1) ? chi2 / (nused - 1) : 0.0;
  out[3] = nused;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Trace and direct evaluation (for parity tests).                             */
/* ------------------------------------------------------------------------ */
int orc_trace(const orc_state* s, int64_t n_points, int64_t iteration, int64_t first,
              int64_t count, int32_t n_words, uint32_t* words, int32_t* chan, int32_t* bins,
              uint8_t* near, double* p, double* fgw) {
  const int K = s->K, d = s->d;
  if (n_words < 0 || n_words > 36) return -1;
  int64_t* nc = (int64_t*)malloc(sizeof(int64_t) * K);
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (K + 1));
  double* alpha = (double*)malloc(sizeof(double) * K);
  int64_t* nr = (int64_t*)calloc(K, sizeof(int64_t));
  int64_t* spb = (int64_t*)calloc(K, sizeof(int64_t));
  orc_allocation(K, s->alpha, n_points, s->min_calls, nc, alpha);
  if (s->strat) strat_adjust(K, d, s->strat, nc, nr, spb, alpha);
  start[0] = 0;
  for (int c = 0; c < K; ++c) start[c + 1] = start[c] + nc[c];
  /* evaluate with the allocated alpha, as the pass itself does */
  orc_state tmp = *s;
  tmp.alpha = alpha;
  uint32_t u[32];
  int rc = 0;
  for (int64_t q = 0; q < count; ++q) {
    const int64_t i = first + q;
    if (i < 0 || i >= start[K]) {
      rc = -1;
      break;
    }
    const int c = channel_of(start, K, i);
    const int nw = n_words > d ? n_words : d;
    uint32_t all[40];
    if (s->rng)
      mrg_call_words(s->seed, c, (uint64_t)(i - start[c]), (uint32_t)iteration, nw, all);
    else
      for (int m = 0; m < nw; ++m)
        all[m] = orc_word(s->seed, (uint64_t)i, (uint32_t)iteration, (uint32_t)m);
    for (int m = 0; m < n_words; ++m) words[q * n_words + m] = all[m];
    for (int m = 0; m < d; ++m) u[m] = all[m];
    int jin[32];
    double fin[32];
    call_bins(s, nr, spb, c, i - start[c], u, jin, fin);
    const point_result r =
        eval_point(&tmp, c, jin, fin, NULL, bins + q * K * d, near + q * K * d, p + q * d);
    chan[q] = c;
    fgw[q * 3 + 0] = r.f;
    fgw[q * 3 + 1] = r.g;
    fgw[q * 3 + 2] = r.w;
  }
  free(nc);
  free(start);
  free(alpha);
  free(nr);
  free(spb);
  return rc;
}

int orc_eval_fg(const orc_state* s, int64_t n, const double* p, double* f, double* g) {
  const int K = s->K, d = s->d, nb = s->n;
  for (int64_t q = 0; q < n; ++q) {
    const double* pp = p + q * d;
    f[q] = integrand(s, pp);
    double gs = 0.0;
    for (int c = 0; c < K; ++c) {
      double qd = 1.0, gc = 1.0;
      for (int k = 0; k < d; ++k) {
        const map1d* m = &s->maps[c * d + k];
        qd *= map_density(m, pp[k]);
        const double* e = EDGE(s, c, k);
        const int J = find_bin(e, nb, map_cdf(m, pp[k]));
        gc *= 1.0 / ((double)nb * (e[J + 1] - e[J]));
      }
      gs += s->alpha[c] * gc * qd;
    }
    g[q] = gs;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Unweighting (Sec. 2 eq. efficiency; Sec. 3.3 simulation by importance      */
/* sampling; Sec. 3.5 last paragraph: fixed grids, channel drawn by alpha).  */
/* [R6] channel = interval of floor(u64 N_tot / 2^64) in the prefix offsets. */
/* [R18] w_max starts at the last pass's maximum weight; it is raised only   */
/* between batches of `batch` trials, so decisions do not depend on order.   */
/* Event generation always samples importance-wise (Sec. 3.3: unweighted     */
/* events must be independent), also after stratified integration passes.   */
/* [R27] Weights may be negative (Sec. 3.1: an NLO integrand need not be     */
/* positive semidefinite): a trial is kept with probability |w| / w_max, w_max */
/* is the largest |w|, and a kept event carries the sign of its weight.      */
/* ------------------------------------------------------------------------ */
/* The unweighting loop.  tie_rel: the relative distance from a threshold
 * within which a decision counts as a tie (another rounding of w could flip
 * it); first_tie_out (may be NULL): the events kept before the first tied
 * decision among the trials up to the last event kept (n_events if none). */
static int unweight_impl(orc_state* s, int64_t n_events, int64_t batch, double tie_rel,
                         double* events, int8_t* signs, double* stats, int64_t* first_tie_out) {
  if (s->n_iter == 0) return -4;
  if (batch < 1) return -1;
  const int K = s->K, d = s->d;
  if (s->ntot == 0) return -4;
  /* The channel is drawn with probability N_c / N_tot, so alpha in g(p) must
   * be that same ratio: re-allocate if alpha moved since the last pass. */
  if (!s->alloc_valid) orc_allocate(s, s->last_n);
  if (s->wmax_unw < 0.0) s->wmax_unw = s->history[(s->n_iter - 1) * 5 + 3];
  double wmax_b = s->wmax_unw;
  int64_t got = 0, n_over = 0, q = s->trials_done, last_used = s->trials_done - 1;
  /* decisions within 1e-12 (relative) of their threshold, which another
   * rounding of w could flip: accepts (u w_max vs w) up to the last event
   * kept, and overweight flags (w vs w_max) of the events kept */
  int64_t accept_ties = 0, over_ties = 0, first_tie = -1;
  uint32_t u[36];
  double p[32];
  while (got < n_events) {
    double bmax = wmax_b;
    for (int64_t b = 0; b < batch; ++b, ++q) {
      if (s->rng)
        mrg_trial_words(s->seed, (uint64_t)q, d + 3, u);
      else
        for (int m = 0; m < d + 3; ++m)
          u[m] = orc_word(s->seed, (uint64_t)q, TAG_UNWEIGHT, (uint32_t)m);
      const uint64_t u64 = (uint64_t)u[d] | ((uint64_t)u[d + 1] << 32);
      const int64_t r = (int64_t)(((unsigned __int128)u64 * (unsigned __int128)s->ntot) >> 64);
      const int c = channel_of(s->start, K, r);
      int jin[32];
      double fin[32];
      for (int k = 0; k < d; ++k) bin_frac(u[k], s->n, s->fp32, &jin[k], &fin[k]);
      const point_result pr = eval_point(s, c, jin, fin, NULL, NULL, NULL, p);
      const double w = pr.w;
      if (!isfinite(w)) continue;
      const double aw = fabs(w); /* [R27] signed weights: |w| against w_max */
      if (aw > bmax) bmax = aw;
      const double acc = ((double)u[d + 2] + 0.5) * 0x1p-32;
      if (got < n_events && fabs(acc * wmax_b - aw) <= tie_rel * aw) {
        ++accept_ties;
        if (first_tie < 0) first_tie = got;
      }
      if (got < n_events && acc * wmax_b < aw) {
        for (int k = 0; k < d; ++k) events[(size_t)k * n_events + got] = p[k];
        if (signs) signs[got] = w < 0.0 ? -1 : 1;
        if (aw > wmax_b) ++n_over;
        if (fabs(aw - wmax_b) <= tie_rel * wmax_b) ++over_ties;
        ++got;
        last_used = q;
      }
    }
    wmax_b = bmax;
  }
  const int64_t trials = last_used + 1 - s->trials_done;
  s->trials_done = q;
  s->wmax_unw = wmax_b;
  stats[0] = (double)trials;
  stats[1] = (double)n_over;
  stats[2] = wmax_b;
  stats[3] = trials > 0 ? (double)n_events / (double)trials : 0.0;
  stats[4] = (double)over_ties;
  stats[5] = (double)accept_ties;
  if (first_tie_out) *first_tie_out = first_tie < 0 ? n_events : first_tie;
  return 0;
}

int orc_unweight_ex(orc_state* s, int64_t n_events, int64_t batch, double* events,
                    int8_t* signs, double* stats) {
  return unweight_impl(s, n_events, batch, 1e-12, events, signs, stats, NULL);
}

int orc_unweight_tol(orc_state* s, int64_t n_events, int64_t batch, double tie_rel,
                     double* events, int8_t* signs, double* stats, int64_t* first_tie) {
  return unweight_impl(s, n_events, batch, tie_rel, events, signs, stats, first_tie);
}

int orc_unweight(orc_state* s, int64_t n_events, int64_t batch, double* events, double* stats) {
  double st[6];
  const int rc = orc_unweight_ex(s, n_events, batch, events, NULL, st);
  if (rc == 0) memcpy(stats, st, 4 * sizeof(double));
  return rc;
}

/* ------------------------------------------------------------------------ */
/* State access                                                               */
/* ------------------------------------------------------------------------ */
int orc_get_edges(const orc_state* s, double* e) {
  memcpy(e, s->edges, sizeof(double) * s->K * s->d * (s->n + 1));
  return 0;
}
int orc_set_edges(orc_state* s, const double* e) {
  memcpy(s->edges, e, sizeof(double) * s->K * s->d * (s->n + 1));
  return 0;
}
int orc_get_alpha(const orc_state* s, double* a) {
  memcpy(a, s->alpha, sizeof(double) * s->K);
  return 0;
}
int orc_set_alpha(orc_state* s, const double* a) {
  memcpy(s->alpha, a, sizeof(double) * s->K);
  s->alloc_valid = 0;
  return 0;
}
int orc_get_alloc(const orc_state* s, int64_t* nc) {
  memcpy(nc, s->nc, sizeof(int64_t) * s->K);
  nc[s->K] = s->ntot;
  return 0;
}
int orc_get_hist(const orc_state* s, double* h) {
  memcpy(h, s->hist, sizeof(double) * s->K * s->d * s->n);
  return 0;
}
int orc_get_channel_stats(const orc_state* s, double* st) {
  for (int c = 0; c < s->K; ++c) {
    st[c * 7 + 0] = s->s1[c];
    st[c * 7 + 1] = s->s2[c];
    st[c * 7 + 2] = s->wmax_c[c];
    st[c * 7 + 3] = (double)s->nbad_c[c];
    st[c * 7 + 4] = s->e_c[c];
    st[c * 7 + 5] = s->w_c[c];
    st[c * 7 + 6] = s->v_c[c];
  }
  return 0;
}
int32_t orc_n_iterations(const orc_state* s) { return s->n_iter; }
int orc_get_history(const orc_state* s, double* h) {
  memcpy(h, s->history, sizeof(double) * 5 * s->n_iter);
  return 0;
}
double orc_wmax(const orc_state* s) { return s->wmax_unw; }
void orc_set_wmax(orc_state* s, double w) { s->wmax_unw = w; }
