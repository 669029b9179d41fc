/*
 * CPU oracle for the Monte Carlo dust radiative transfer path.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 reference implementation used
 * by the tests, by the smoke check and by the CPU baseline of the benchmark.
 * The product path never includes, links or calls anything in this directory.
 *
 * Method (paper, Sec. 2 "Monte Carlo method"): a point star emits photon
 * packets of constant energy eps at frequencies drawn from its spectrum; a
 * packet flies cell by cell through a grid of cubes and subcubes; the chance
 * of an interaction in a cell follows from the extinction optical depth along
 * the path; on scattering only the direction changes (phase function); on
 * absorption the cell gains eps and a new packet of the same energy is emitted
 * isotropically from the same spot at a new frequency chosen from the cell
 * temperature *before* the absorption (the simplified re-emission law that
 * allows parallel flights).  Transiently heated PAHs (Sec. 1, Sec. 4, Fig. 3)
 * are handled by a steady-state enthalpy-bin solver for P(T).
 */
#ifndef MCRT_ORACLE_H
#define MCRT_ORACLE_H
#include <stdint.h>

#define ORC_FLAG_TALLY_J        1
#define ORC_FLAG_FROZEN_T       2
#define ORC_FLAG_KILL_ON_ABSORB 4
#define ORC_FLAG_EXACT_BW        8
#define ORC_FLAG_PEEL           16
#define ORC_FLAG_PEEL_SED       32   /* with PEEL: next-event SED per observer, every bin */

enum {
  ORC_CNT_LAUNCHED = 0, ORC_CNT_ESCAPED, ORC_CNT_KILLED, ORC_CNT_TERMINATED,
  ORC_CNT_SCATTERS, ORC_CNT_ABSORPTIONS, ORC_CNT_CROSSINGS, ORC_CNT_TCLAMP_LO,
  ORC_CNT_TCLAMP_HI, ORC_CNT_PAH_ABS, ORC_CNT_ZERO_CROSS, ORC_CNT_JSEG, ORC_CNT_PEEL,
  ORC_N_COUNTERS = 16
};

enum { ORC_EV_LAUNCH = 0, ORC_EV_CROSS = 1, ORC_EV_SCATTER = 2, ORC_EV_ABSORB = 3,
       ORC_EV_ESCAPE = 4, ORC_EV_KILLED = 5 };

typedef struct {
  int32_t type, cell, j, pad;
  double x[3], d[3], tau;          /* x in base-cube units */
} orc_trace_rec;

typedef struct {
  /* spectrum and species */
  int32_t nl, S;
  const double *lam_um;            /* [nl] */
  const double *kabs, *ksca;       /* [S*nl], cm^2 per gram of mixture */
  const double *g;                 /* [nl] */
  const int32_t *kind;             /* [S] 0 equilibrium, 1 PAH */
  /* grid */
  int32_t nb, L;
  int64_t n_cells, n_nodes;
  double box_min[3], base_size;
  const int32_t *base_map, *nodes;
  const double *rho;               /* [n_cells], g cm^-3 */
  /* source */
  double src_pos[3], lum, teff, beam[3];
  int32_t beam_on;
  /* temperature grid */
  int32_t K;
  double T_lo, T_hi;
  /* run */
  uint64_t n_total, seed, max_events;
  int32_t n_theta, n_phi;
  int32_t flags;
  int32_t n_threads;               /* 1 = sequential definition */
  const uint64_t *frozen_nabs;     /* [n_cells*S] (frozen_T mode) */
  const double *pah_rows;          /* [n_pah][n_cells][nl] CDF rows or NULL */
  /* escape images (n_obs = 0: none) */
  int32_t n_obs, npix, n_img_lambda, pad_img;
  int32_t img_lambda[8];           /* imaged wavelength bins */
  double img_center[3];            /* cm */
  double img_half_width;           /* cm */
  double img_cos_cone;             /* in (0, 1] */
  double obs_dir[8][3];            /* towards the observers (normalised here) */
  /* optional: row of (PAH slot p, cell c) is pah_rows + pah_row_map[p n_cells + c] nl,
     so many cells can share a row of a compact table; NULL = the dense layout */
  const int32_t *pah_row_map;      /* [n_pah][n_cells] or NULL */
} orc_problem;

typedef struct {
  double *nu, *dnu;                /* [nl] */
  double *src_cdf;                 /* [nl] */
  double *kext, *albedo;           /* [nl] cm^2 g^-1, - */
  double *sp_cdf;                  /* [nl*S] */
  double *Tk;                      /* [K] */
  double *E;                       /* [S*K] erg s^-1 g^-1 */
  double *R;                       /* [S*(K-1)*nl] */
} orc_tables;

typedef struct {
  uint64_t *nabs;                  /* [n_cells*S] */
  uint64_t *sed;                   /* [n_theta*n_phi*nl] */
  uint64_t *jq;                    /* [nl*n_cells] fixed-point path sums or NULL */
  uint64_t *counters;              /* [16] */
  uint64_t *image;                 /* [n_obs*n_img_lambda*npix*npix] or NULL */
  orc_trace_rec *trace;            /* [n*trace_cap] or NULL */
  int32_t *trace_len;              /* [n] */
  int64_t trace_cap;
  uint64_t *peel;                  /* [n_obs*n_img_lambda*npix*npix] next-event
                                      weights, fixed point 2^-24, or NULL */
  uint64_t *peel_sed;              /* [n_obs*nl] next-event SED per observer
                                      (ORC_FLAG_PEEL_SED), fixed point 2^-24, or NULL */
} orc_out;

#ifdef __cplusplus
extern "C" {
#endif
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u24(uint32_t w);
double orc_planck_nu(double nu, double T);
void orc_lambda_bins(int32_t nl, const double *lam_um, double *nu, double *dnu);
void orc_build_tables(const orc_problem *p, orc_tables *t);
int orc_locate(const orc_problem *p, const int64_t F[3], int32_t *level, int64_t lo[3]);
int orc_transport(const orc_problem *p, const orc_tables *t, uint64_t first_id,
                  uint64_t n, orc_out *o);
void orc_temperatures(const orc_problem *p, const orc_tables *t, const uint64_t *nabs,
                      double *T_out);
void orc_mean_intensity(const orc_problem *p, const orc_tables *t, const uint64_t *jq,
                        double *J_out);
/* PAH steady state (per cell): see the implementation. */
void orc_pah_solve(int32_t M, const double *T, const double *U, int32_t nl,
                   const double *lam_um, const double *cabs, const double *cband,
                   int32_t n_bands, const double *ccont, const double *J, int64_t n,
                   double *out, double *P_out, double *pabs_out, int32_t n_threads);
void orc_pah_rates(int32_t M, const double *T, const double *U, int32_t nl,
                   const double *lam_um, const double *cabs, const double *J,
                   double *A_up, double *A_down);
void orc_thin_field(const orc_problem *p, const orc_tables *t, double *J_out);
void orc_pah_rows(int32_t nl, int32_t n_bands, const double *lam_um, const double *cband,
                  const double *out, int64_t n, double *rows);
#ifdef __cplusplus
}
#endif
#endif
