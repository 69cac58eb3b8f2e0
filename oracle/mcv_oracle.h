/*
 * FP64 CPU oracle for the multi-channel VEGAS (VAMP) sample pass.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library: the only thing both sides see is the problem description produced
 * by the seeded input generators.
 *
 * Every function follows a passage of Brass, Kilian, Reuter, "Parallel
 * Adaptive Monte Carlo Integration with the Event Generator WHIZARD"
 * (arXiv:1811.09711); the citation sits on each definition in mcv_oracle.c.
 */
#ifndef MCV_ORACLE_H
#define MCV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FLAT = 0, ORC_GAUSS = 1, ORC_BW = 2 };
enum { ORC_REFINE_GRID = 1, ORC_REFINE_ALPHA = 2 };

typedef struct {
  int32_t dim, n_channels, n_bins, n_peaks;
  int32_t fp32_rules;          /* 1: precision-mode rules (24-bit fraction, FP32-snapped edges) */
  const int32_t* peak_kind;    /* [P*d] */
  const double* peak_loc;      /* [P*d] */
  const double* peak_width;    /* [P*d] sigma (Gauss) or FWHM (BW) */
  const double* peak_weight;   /* [P] */
  const int32_t* chan_kind;    /* [K*d] */
  const double* chan_loc;      /* [K*d] */
  const double* chan_width;    /* [K*d] */
  uint64_t seed;
  double grid_power;           /* exponent of the bin measure m_j */
  double channel_power;        /* exponent beta of the channel-weight update */
  int64_t min_calls;           /* floor on N_c */
  int32_t rng;                 /* 0: Philox4x32-10 words; 1: MRG32k3a streams (K <= 1023,
                                  seed < 2^54) */
  int32_t strat;               /* 0: uniform r (importance sampling); s >= 2: pseudo-stratified
                                  in r space, at least s calls per box */
} orc_problem;

typedef struct orc_state orc_state;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Word m of sample i at iteration tag t: output (m mod 4) of the block with
 * counter (i_lo, i_hi, t, m/4) and key (seed_lo, seed_hi). */
uint32_t orc_word(uint64_t seed, uint64_t i, uint32_t t, uint32_t m);

/* MRG32k3a: `count` outputs z (in [1, m1]) of substream i of stream g,
 * starting `offset` steps in, from the all-12345 initial state. */
void orc_mrg_outputs(uint64_t g, uint64_t i, uint64_t offset, int32_t count, uint32_t* z);

double orc_erfcinv(double y);
/* 1-d maps: kind, loc, width; x in (0,1) -> p; p -> x (CDF); density q(p). */
double orc_map_forward(int32_t kind, double loc, double width, double x);
double orc_map_cdf(int32_t kind, double loc, double width, double p);
double orc_map_density(int32_t kind, double loc, double width, double p);
double orc_peak_pdf(int32_t kind, double loc, double width, double p);

orc_state* orc_create(const orc_problem* prob, int32_t max_iter);
void orc_destroy(orc_state* s);

/* Stratified layout of a channel with n calls in d dimensions, at least
 * s_min calls per box: boxes per axis nr (the largest with s_min nr^d <= n,
 * at most 2^20) and calls per box floor(n / nr^d). */
void orc_strat_layout(int64_t n, int32_t d, int64_t s_min, int64_t* nr, int64_t* per_box);

/* Channel allocation N_c from alpha and n_points; sets alpha_c = N_c/N_tot. */
int orc_allocate(orc_state* s, int64_t n_points);
/* One integration pass at the current iteration index; n_threads >= 1. */
int orc_sample_iteration(orc_state* s, int64_t n_points, int32_t n_threads);
int orc_refine(orc_state* s, uint32_t what);
/* out: integral, error, chi2/ndf, iterations used */
int orc_result(const orc_state* s, int32_t first_iter, double out[4]);

/* Per-point trace of the pass with n_points at iteration index `iteration`
 * (state is not modified).  bins: [count][K][d] (own channel: own bins),
 * near: [count][K][d] 1 where an other-channel coordinate lies within 1e-12 of
 * a bin edge, words: [count][n_words], p: [count][d], fgw: [count][3]. */
int orc_trace(const orc_state* s, int64_t n_points, int64_t iteration, int64_t first,
              int64_t count, int32_t n_words, uint32_t* words, int32_t* chan,
              int32_t* bins, uint8_t* near, double* p, double* fgw);

/* f(p) and g(p) at arbitrary points p[n][d] with the current grids and alpha. */
int orc_eval_fg(const orc_state* s, int64_t n, const double* p, double* f, double* g);

/* Rejection unweighting with fixed grids.  events: [d][n_events];
 * stats: trials, n_overweight, final w_max, efficiency. */
int orc_unweight(orc_state* s, int64_t n_events, int64_t batch, double* events,
                 double* stats);
/* The same, with the sign of each kept event's weight (signs [n_events], may
 * be NULL) and stats[6]: the four above, then the number of kept events whose
 * |w| lies within 1e-12 (relative) of the batch's w_max (an overweight flag
 * another rounding of w could flip), and the number of trials up to the last
 * kept one whose accept test lies within 1e-12 of |w|. */
int orc_unweight_ex(orc_state* s, int64_t n_events, int64_t batch, double* events,
                    int8_t* signs, double* stats);
/* orc_unweight_ex with decisions within tie_rel (relative) of their
 * threshold counted as ties (stats[4], stats[5]); *first_tie: the events
 * kept before the first tied accept decision (n_events if none).  For
 * comparisons with weights that carry more rounding (FP32 mode). */
int orc_unweight_tol(orc_state* s, int64_t n_events, int64_t batch, double tie_rel,
                     double* events, int8_t* signs, double* stats, int64_t* first_tie);

/* State access (host copies). */
int orc_get_edges(const orc_state* s, double* edges);     /* [K][d][n+1] */
int orc_set_edges(orc_state* s, const double* edges);
int orc_get_alpha(const orc_state* s, double* alpha);     /* [K] */
int orc_set_alpha(orc_state* s, const double* alpha);
int orc_get_alloc(const orc_state* s, int64_t* nc);       /* [K+1]: N_c..., N_tot */
int orc_get_hist(const orc_state* s, double* hist);       /* [K][d][n] */
/* per channel: S1, S2, wmax, nbad, E_c, W_c, V_c  -> [K][7] */
int orc_get_channel_stats(const orc_state* s, double* stats);
int32_t orc_n_iterations(const orc_state* s);
/* per iteration: E, sigma, N_tot, wmax, nbad -> [n_iter][5] */
int orc_get_history(const orc_state* s, double* hist);
/* Rebin one axis: n old edges + histogram -> new edges (for pins). */
int orc_rebin_axis(int32_t n, const double* edges, const double* hist, double power,
                   int32_t snap32, double* out_edges);
int orc_update_alpha(int32_t K, double* alpha, const double* w2, double beta);
/* Channel equivalences applied before every grid rebinning: eq [n_eq][2 + 2d]
 * = c, c', perm[d] (axis of c' for each axis of c, a permutation), mode[d]
 * (0 identity, 1 invert, 2 symmetric, 3 invariant).  n_eq = 0 clears them.
 * Returns -1 (and keeps the old list) for a malformed list. */
int orc_set_equivalences(orc_state* s, int32_t n_eq, const int32_t* eq);
/* The per-bin weights after the equivalences, [K][d][n] (for pins). */
int orc_get_equivalent_hist(const orc_state* s, double* out);
int orc_allocation(int32_t K, const double* alpha, int64_t n_points, int64_t min_calls,
                   int64_t* nc, double* alpha_out);
double orc_wmax(const orc_state* s);
void orc_set_wmax(orc_state* s, double w);

#ifdef __cplusplus
}
#endif
#endif
