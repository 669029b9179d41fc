/*
 * CPU oracle for the Monte Carlo dust radiative transfer path, FP64.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests/, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP engine.
 *
 * Sections of the paper followed:
 *   Sec. 2  packets of constant energy from the star, extinction optical depth
 *           per cell, scattering by the phase function, absorption raising the
 *           cell energy by eps and isotropic re-emission at a new frequency
 *           chosen from the temperature before the absorption, grid of cubes
 *           and subcubes;
 *   Sec. 1  grain and PAH cross-sections, 17 Lorentzian PAH bands;
 *   Fig. 3 / Sec. 4  temperature distribution P(T) of transiently heated PAHs.
 * Where the paper is silent the readings listed in the design notes apply
 * (wavelength bins with constant cross-sections, Philox random streams keyed
 * by packet id, tie rules at cell faces, difference-emissivity rows).
 */
#include "mcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double C_LIGHT = 2.99792458e10;   /* cm s^-1 */
static const double H_PLANCK = 6.62607015e-27; /* erg s */
static const double K_BOLTZ = 1.380649e-16;    /* erg K^-1 */
static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw 2011):  */
/* each round multiplies words 0 and 2 by the two round multipliers, splits   */
/* the 64-bit products into high/low halves, and mixes them with the other    */
/* two words and the key; the key is bumped by the two Weyl constants between */
/* rounds.  Ten rounds.                                                       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform on (0,1]: the top 24 bits plus one, times 2^-24 (exact in FP32) */
double orc_u24(uint32_t w) { return (double)((w >> 8) + 1u) * (1.0 / 16777216.0); }

/* eight uniforms of event slot e of packet pid */
static void draw_slot(uint64_t seed, uint64_t pid, uint32_t e, double u[8]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t c[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), e, 0u}, w[4];
  orc_philox4x32_10(c, key, w);
  for (int i = 0; i < 4; ++i) u[i] = orc_u24(w[i]);
  c[3] = 1u;
  orc_philox4x32_10(c, key, w);
  for (int i = 0; i < 4; ++i) u[4 + i] = orc_u24(w[i]);
}

/* ------------------------------------------------------------------------ */
/* spectra                                                                    */
/* ------------------------------------------------------------------------ */
double orc_planck_nu(double nu, double T) {
  double x = H_PLANCK * nu / (K_BOLTZ * T);
  return 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT) / expm1(x);
}

/* Frequencies of the bin centres and bin widths.  Bin edges lie at the
 * geometric midpoints of neighbouring wavelengths; the outer edges half a
 * logarithmic step beyond the first and last centre. */
void orc_lambda_bins(int32_t nl, const double *lam_um, double *nu, double *dnu) {
  for (int j = 0; j < nl; ++j) {
    double lam = lam_um[j] * 1e-4;
    double lo, hi; /* wavelength edges in cm */
    if (j > 0) lo = sqrt(lam_um[j - 1] * lam_um[j]) * 1e-4;
    else lo = lam_um[0] * lam_um[0] / sqrt(lam_um[0] * lam_um[1]) * 1e-4;
    if (j < nl - 1) hi = sqrt(lam_um[j] * lam_um[j + 1]) * 1e-4;
    else hi = lam_um[nl - 1] * lam_um[nl - 1] / sqrt(lam_um[nl - 2] * lam_um[nl - 1]) * 1e-4;
    nu[j] = C_LIGHT / lam;
    dnu[j] = C_LIGHT / lo - C_LIGHT / hi;
  }
}

/* Tables: source spectrum CDF over bins, extinction and albedo per bin,
 * species choice CDF per bin, emission E_s(T_k) = 4 pi sum_j kabs B dnu, and
 * the difference-emissivity rows R_{s,k}: CDF over j of kabs_s(j)
 * [B_j(T_{k+1}) - B_j(T_k)] dnu_j, i.e. the spectrum in which a grain at
 * T_k gives out the energy of one more absorbed packet. */
void orc_build_tables(const orc_problem *p, orc_tables *t) {
  const int nl = p->nl, S = p->S, K = p->K;
  orc_lambda_bins(nl, p->lam_um, t->nu, t->dnu);
  double tot = 0.0;
  for (int j = 0; j < nl; ++j) { tot += orc_planck_nu(t->nu[j], p->teff) * t->dnu[j]; t->src_cdf[j] = tot; }
  for (int j = 0; j < nl; ++j) t->src_cdf[j] /= tot;
  t->src_cdf[nl - 1] = 1.0;
  for (int j = 0; j < nl; ++j) {
    double ka = 0.0, ks = 0.0;
    for (int s = 0; s < S; ++s) { ka += p->kabs[s * nl + j]; ks += p->ksca[s * nl + j]; }
    t->kext[j] = ka + ks;
    t->albedo[j] = (ka + ks) > 0.0 ? ks / (ka + ks) : 0.0;
    double cum = 0.0;
    for (int s = 0; s < S; ++s) {
      cum += p->kabs[s * nl + j];
      t->sp_cdf[j * S + s] = ka > 0.0 ? cum / ka : 1.0;
    }
    t->sp_cdf[j * S + S - 1] = 1.0;
  }
  for (int k = 0; k < K; ++k) t->Tk[k] = p->T_lo * pow(p->T_hi / p->T_lo, (double)k / (double)(K - 1));
  for (int s = 0; s < S; ++s) {
    for (int k = 0; k < K; ++k) {
      double e = 0.0;
      for (int j = 0; j < nl; ++j) e += p->kabs[s * nl + j] * orc_planck_nu(t->nu[j], t->Tk[k]) * t->dnu[j];
      t->E[s * K + k] = 4.0 * PI * e;
    }
    for (int k = 0; k < K - 1; ++k) {
      double *row = t->R + ((int64_t)s * (K - 1) + k) * nl;
      double cum = 0.0;
      for (int j = 0; j < nl; ++j) {
        double dB = orc_planck_nu(t->nu[j], t->Tk[k + 1]) - orc_planck_nu(t->nu[j], t->Tk[k]);
        cum += p->kabs[s * nl + j] * dB * t->dnu[j];
        row[j] = cum;
      }
      for (int j = 0; j < nl; ++j) row[j] = cum > 0.0 ? row[j] / cum : 1.0;
      row[nl - 1] = 1.0;
    }
  }
}

/* first index j in [0,n) with cdf[j] >= u (cdf[n-1] == 1 >= u) */
static int cdf_search(const double *cdf, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* ------------------------------------------------------------------------ */
/* grid: base cubes and subcubes (Sec. 2)                                     */
/* ------------------------------------------------------------------------ */
/* Leaf containing the finest-unit integer point F; returns the cell id, its
 * level and lower corner in finest units, or -1 when F is outside the grid. */
int orc_locate(const orc_problem *p, const int64_t F[3], int32_t *level, int64_t lo[3]) {
  const int L = p->L;
  const int64_t nf = (int64_t)1 << L, ext = (int64_t)p->nb * nf;
  for (int a = 0; a < 3; ++a)
    if (F[a] < 0 || F[a] >= ext) return -1;
  int64_t b[3] = {F[0] >> L, F[1] >> L, F[2] >> L};
  int32_t e = p->base_map[b[0] + (int64_t)p->nb * (b[1] + (int64_t)p->nb * b[2])];
  int lev = 0;
  while (e < 0) {
    int node = -e - 1;
    lev += 1;
    int sh = L - lev;
    int o = (int)((F[0] >> sh) & 1) | (int)(((F[1] >> sh) & 1) << 1) | (int)(((F[2] >> sh) & 1) << 2);
    e = p->nodes[(int64_t)node * 8 + o];
  }
  *level = lev;
  int sh = L - lev;
  for (int a = 0; a < 3; ++a) lo[a] = (F[a] >> sh) << sh;
  return e;
}

/* ------------------------------------------------------------------------ */
/* packet transport                                                           */
/* ------------------------------------------------------------------------ */
static void iso_dir(double mu, double phi, double d[3]) {
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  d[0] = st * cos(phi); d[1] = st * sin(phi); d[2] = mu;
}

/* Henyey-Greenstein (1941) deflection cosine by inversion of its CDF */
static double hg_mu(double g, double u) {
  if (fabs(g) < 1e-5) return 2.0 * u - 1.0;
  double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
  double mu = (1.0 + g * g - f * f) / (2.0 * g);
  return fmin(1.0, fmax(-1.0, mu));
}

/* turn d by polar angle acos(mu) and azimuth phi about itself
 * (direction-cosine update; near the poles the frame is the lab frame) */
static void rotate_dir(double d[3], double mu, double phi) {
  double st = sqrt(fmax(0.0, 1.0 - mu * mu)), cp = cos(phi), sp = sin(phi);
  double ux = d[0], uy = d[1], uz = d[2];
  if (fabs(uz) > 0.99999) {
    d[0] = st * cp; d[1] = st * sp; d[2] = (uz >= 0.0 ? mu : -mu);
    return;
  }
  double tmp = sqrt(1.0 - uz * uz);
  d[0] = st * (ux * uz * cp - uy * sp) / tmp + ux * mu;
  d[1] = st * (uy * uz * cp + ux * sp) / tmp + uy * mu;
  d[2] = -st * cp * tmp + uz * mu;
}

static inline uint64_t add_u64(uint64_t *a, uint64_t v, int threaded) {
  if (threaded) return __atomic_fetch_add(a, v, __ATOMIC_RELAXED);
  uint64_t old = *a; *a = old + v; return old;
}

static void rec(orc_out *o, uint64_t k, int type, int cell, int j, const double x[3],
                const double d[3], double tau) {
  if (!o->trace) return;
  int32_t n = o->trace_len[k];
  if (n >= o->trace_cap) return;
  orc_trace_rec *r = o->trace + (int64_t)k * o->trace_cap + n;
  r->type = type; r->cell = cell; r->j = j; r->pad = 0;
  for (int a = 0; a < 3; ++a) { r->x[a] = x[a]; r->d[a] = d[a]; }
  r->tau = tau;
  o->trace_len[k] = n + 1;
}

static void escape_tally(const orc_problem *p, orc_out *o, const double d[3], int j, int thr) {
  int bt = (int)floor((d[2] + 1.0) * 0.5 * p->n_theta);
  if (bt < 0) bt = 0;
  if (bt >= p->n_theta) bt = p->n_theta - 1;
  double phi = atan2(d[1], d[0]);
  if (phi < 0.0) phi += 2.0 * PI;
  int bp = (int)floor(phi / (2.0 * PI) * p->n_phi);
  if (bp < 0) bp = 0;
  if (bp >= p->n_phi) bp = p->n_phi - 1;
  add_u64(&o->sed[((int64_t)bt * p->n_phi + bp) * p->nl + j], 1, thr);
}

/* Escape images: observer o looks back along n_o (unit).  A packet leaving
 * the grid at x (base-cube units) in direction d with d . n_o >= cos_cone,
 * in an imaged bin, is placed where its ray, extended backwards, crosses the
 * image plane through the centre c perpendicular to n_o; the plane's axes are
 * e1 = (z x n_o)/|z x n_o| (the x axis when n_o is along z) and
 * e2 = n_o x e1; pixel (px, py) = floor((a + w) / (2 w) npix) of the plane
 * coordinates (a, b), counted when both lie in [0, npix). */
static void image_tally(const orc_problem *p, orc_out *o, const double x[3], const double d[3],
                        int j, int thr) {
  if (!o->image || p->n_obs <= 0) return;
  int l = -1;
  for (int q = 0; q < p->n_img_lambda; ++q) if (p->img_lambda[q] == j) l = q;
  if (l < 0) return;
  double X[3];                                       /* exit point relative to c, cm */
  for (int a = 0; a < 3; ++a) X[a] = p->box_min[a] + x[a] * p->base_size - p->img_center[a];
  for (int ob = 0; ob < p->n_obs; ++ob) {
    const double *m = p->obs_dir[ob];
    const double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    const double n[3] = {m[0] / len, m[1] / len, m[2] / len};
    const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    if (dn < p->img_cos_cone) continue;
    double e1[3], e2[3];
    const double r = sqrt(n[0] * n[0] + n[1] * n[1]);
    if (r > 1e-12) { e1[0] = -n[1] / r; e1[1] = n[0] / r; e1[2] = 0.0; }
    else { e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0; }
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];
    /* back along the ray to the plane X . n = 0 */
    const double s = (X[0] * n[0] + X[1] * n[1] + X[2] * n[2]) / dn;
    double P[3];
    for (int a = 0; a < 3; ++a) P[a] = X[a] - s * d[a];
    const double ca = P[0] * e1[0] + P[1] * e1[1] + P[2] * e1[2];
    const double cb = P[0] * e2[0] + P[1] * e2[1] + P[2] * e2[2];
    const double w = p->img_half_width;
    const double fx = floor((ca + w) / (2.0 * w) * p->npix), fy = floor((cb + w) / (2.0 * w) * p->npix);
    if (fx < 0.0 || fy < 0.0 || fx >= p->npix || fy >= p->npix) continue;
    add_u64(&o->image[(((int64_t)ob * p->n_img_lambda + l) * p->npix + (int64_t)fy) * p->npix + (int64_t)fx],
            1, thr);
  }
}

/* Henyey-Greenstein phase function normalised to a mean of 1 over the sphere:
 * (1 - g^2) / (1 + g^2 - 2 g mu)^(3/2); isotropic below |g| = 1e-5, as the
 * deflection sampler. */
static double hg_phase(double g, double mu) {
  if (fabs(g) < 1e-5) return 1.0;
  const double den = 1.0 + g * g - 2.0 * g * mu;
  return (1.0 - g * g) / (den * sqrt(den));
}

/* Optical depth at bin j from x (base-cube units, inside leaf `cell` of
 * depth lev and lower corner lo) along unit n to the edge of the grid, cell
 * by cell with the transport's own face rules. */
static double peel_tau(const orc_problem *p, const orc_tables *t, const double x0[3], int cell,
                       int lev, const int64_t lo0[3], int j, const double n[3]) {
  const int L = p->L;
  const int64_t nf = (int64_t)1 << L;
  const double h = p->base_size;
  double x[3] = {x0[0], x0[1], x0[2]}, tau = 0.0;
  int64_t lo[3] = {lo0[0], lo0[1], lo0[2]};
  for (;;) {
    const double side = ldexp(1.0, -lev);
    double tex = INFINITY;
    int ax = -1;
    for (int a = 0; a < 3; ++a) {
      const double boxlo = (double)lo[a] / (double)nf;
      double ta;
      if (n[a] > 0.0) ta = (boxlo + side - x[a]) / n[a];
      else if (n[a] < 0.0) ta = (boxlo - x[a]) / n[a];
      else continue;
      if (ta < 0.0) ta = 0.0;
      if (ta < tex) { tex = ta; ax = a; }
    }
    tau += p->rho[cell] * t->kext[j] * h * tex;
    for (int a = 0; a < 3; ++a) x[a] += tex * n[a];
    const int64_t span = (int64_t)1 << (L - lev);
    x[ax] = (double)(n[ax] > 0.0 ? lo[ax] + span : lo[ax]) / (double)nf;
    int64_t G[3];
    for (int a = 0; a < 3; ++a) {
      if (a == ax) G[a] = n[a] > 0.0 ? lo[a] + span : lo[a] - 1;
      else {
        int64_t f = (int64_t)floor(x[a] * (double)nf);
        if (f < lo[a]) f = lo[a];
        if (f > lo[a] + span - 1) f = lo[a] + span - 1;
        G[a] = f;
      }
    }
    cell = orc_locate(p, G, &lev, lo);
    if (cell < 0) return tau;
  }
}

/* Next-event (peel-off) images: at every emission (the star's, unless it
 * is a pencil beam; a re-emission after absorption) and every scattering in
 * an imaged bin, each
 * observer receives the packet's chance per unit solid angle of leaving
 * towards it, times 4 pi: 1 for isotropic emission, hg_phase(g, din . n) for
 * a scattering of a packet that arrived along din; times exp(-tau) of the
 * path from the event to the grid edge along n.  The weight is added in
 * fixed point (round to nearest of 2^24 w) at the pixel of the event's
 * projection on the image plane (the escape images' axes and pixels).  The
 * flux of a pixel at distance D is eps / (4 pi D^2) 2^-24 times its sum. */
static void peel_tally(const orc_problem *p, const orc_tables *t, orc_out *o, const double x[3],
                       int cell, int lev, const int64_t lo[3], int j, const double *din, int thr) {
  if (!o->peel || !(p->flags & ORC_FLAG_PEEL) || p->n_obs <= 0 || cell < 0) return;
  const int sed = (p->flags & ORC_FLAG_PEEL_SED) && o->peel_sed;
  int l = -1;
  for (int q = 0; q < p->n_img_lambda; ++q) if (p->img_lambda[q] == j) l = q;
  if (l < 0 && !sed) return;
  add_u64(&o->counters[ORC_CNT_PEEL], 1, thr);
  double X[3];
  for (int a = 0; a < 3; ++a) X[a] = p->box_min[a] + x[a] * p->base_size - p->img_center[a];
  for (int ob = 0; ob < p->n_obs; ++ob) {
    const double *m = p->obs_dir[ob];
    const double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    const double n[3] = {m[0] / len, m[1] / len, m[2] / len};
    double e1[3], e2[3];
    const double r = sqrt(n[0] * n[0] + n[1] * n[1]);
    if (r > 1e-12) { e1[0] = -n[1] / r; e1[1] = n[0] / r; e1[2] = 0.0; }
    else { e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0; }
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];
    const double ca = X[0] * e1[0] + X[1] * e1[1] + X[2] * e1[2];
    const double cb = X[0] * e2[0] + X[1] * e2[1] + X[2] * e2[2];
    const double w = p->img_half_width;
    const double fx = floor((ca + w) / (2.0 * w) * p->npix), fy = floor((cb + w) / (2.0 * w) * p->npix);
    const int in_img = l >= 0 && !(fx < 0.0 || fy < 0.0 || fx >= p->npix || fy >= p->npix);
    if (!in_img && !sed) continue;
    const double phase = din ? hg_phase(p->g[j], din[0] * n[0] + din[1] * n[1] + din[2] * n[2]) : 1.0;
    const double wgt = phase * exp(-peel_tau(p, t, x, cell, lev, lo, j, n));
    const uint64_t q = (uint64_t)rint(wgt * 16777216.0);
    if (in_img)
      add_u64(&o->peel[(((int64_t)ob * p->n_img_lambda + l) * p->npix + (int64_t)fy) * p->npix + (int64_t)fx],
              q, thr);
    /* the observer's next-event SED: every bin, wherever the event projects */
    if (sed) add_u64(&o->peel_sed[(int64_t)ob * p->nl + j], q, thr);
  }
}

/* One packet from launch to escape / kill.  k indexes the trace buffer. */
static void run_packet(const orc_problem *p, const orc_tables *t, uint64_t pid, uint64_t k,
                       orc_out *o, const int32_t *pah_slot, int thr) {
  const int nl = p->nl, S = p->S, K = p->K, L = p->L;
  const double h = p->base_size;
  const double eps = p->lum / (double)p->n_total;
  const double qscale = ldexp(1.0, L + 16);          /* fixed-point units per base unit */
  const int64_t nf = (int64_t)1 << L;
  uint64_t *cnt = o->counters;
  double u[8];
  draw_slot(p->seed, pid, 0u, u);
  add_u64(&cnt[ORC_CNT_LAUNCHED], 1, thr);
  int j = cdf_search(t->src_cdf, nl, u[0]);
  double d[3];
  if (p->beam_on) { d[0] = p->beam[0]; d[1] = p->beam[1]; d[2] = p->beam[2]; }
  else iso_dir(2.0 * u[1] - 1.0, 2.0 * PI * u[2], d);
  double tau = -log(u[3]);
  double x[3];
  int64_t F[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = (p->src_pos[a] - p->box_min[a]) / h;
    F[a] = (int64_t)floor(x[a] * (double)nf);
  }
  int32_t lev;
  int64_t lo[3];
  int cell = orc_locate(p, F, &lev, lo);
  rec(o, k, ORC_EV_LAUNCH, cell, j, x, d, tau);
  if (!p->beam_on) peel_tally(p, t, o, x, cell, lev, lo, j, NULL, thr);   /* a beam sends nothing sideways */
  if (cell < 0) {
    add_u64(&cnt[ORC_CNT_ESCAPED], 1, thr);
    escape_tally(p, o, d, j, thr);
    image_tally(p, o, x, d, j, thr);
    rec(o, k, ORC_EV_ESCAPE, -1, j, x, d, tau);
    return;
  }
  uint64_t events = 0;
  for (;;) {
    /* exit distance from the current leaf box (lowest axis wins ties) */
    double side = ldexp(1.0, -lev);
    double tex = INFINITY;
    int ax = -1;
    for (int a = 0; a < 3; ++a) {
      double boxlo = (double)lo[a] / (double)nf;
      double ta;
      if (d[a] > 0.0) ta = (boxlo + side - x[a]) / d[a];
      else if (d[a] < 0.0) ta = (boxlo - x[a]) / d[a];
      else continue;
      if (ta < 0.0) ta = 0.0;
      if (ta < tex) { tex = ta; ax = a; }
    }
    double alpha = p->rho[cell] * t->kext[j] * h;      /* extinction per base unit */
    int dusty = p->rho[cell] > 0.0;
    if (alpha > 0.0 && tau < alpha * tex) {
      /* interaction inside this cell */
      double s = tau / alpha;
      for (int a = 0; a < 3; ++a) x[a] += s * d[a];
      if ((p->flags & ORC_FLAG_TALLY_J) && dusty) {
        add_u64(&o->jq[(int64_t)j * p->n_cells + cell], (uint64_t)rint(s * qscale), thr);
        add_u64(&cnt[ORC_CNT_JSEG], 1, thr);
      }
      events += 1;
      if (events > p->max_events) {
        add_u64(&cnt[ORC_CNT_KILLED], 1, thr);
        rec(o, k, ORC_EV_KILLED, cell, j, x, d, tau);
        return;
      }
      draw_slot(p->seed, pid, (uint32_t)events, u);
      if (u[0] <= t->albedo[j]) {
        const double din[3] = {d[0], d[1], d[2]};
        peel_tally(p, t, o, x, cell, lev, lo, j, din, thr);
        rotate_dir(d, hg_mu(p->g[j], u[1]), 2.0 * PI * u[2]);
        add_u64(&cnt[ORC_CNT_SCATTERS], 1, thr);
        tau = -log(u[3]);
        rec(o, k, ORC_EV_SCATTER, cell, j, x, d, tau);
      } else {
        int sp = cdf_search(t->sp_cdf + (int64_t)j * S, S, u[1]);
        uint64_t before = add_u64(&o->nabs[(int64_t)cell * S + sp], 1, thr);
        add_u64(&cnt[ORC_CNT_ABSORPTIONS], 1, thr);
        if (p->flags & ORC_FLAG_FROZEN_T) before = p->frozen_nabs[(int64_t)cell * S + sp];
        if (p->flags & ORC_FLAG_KILL_ON_ABSORB) {
          add_u64(&cnt[ORC_CNT_TERMINATED], 1, thr);
          rec(o, k, ORC_EV_ABSORB, cell, j, x, d, tau);
          return;
        }
        if (p->kind[sp] == 0) {
          /* temperature bracket before this absorption:
           * k = max{k : E_s(T_k) <= N_before eps / (rho V)}, clamped.
           * Exact Bjorkman-Wood form: the new frequency follows
           * kabs [B(T_after) - B(T_before)], with T_before and T_after the
           * temperatures at N_before and N_before + 1 absorptions.  On the
           * table this difference is the sum of the bracket rows between the
           * two, each weighted by the part of [E(T_before), E(T_after)] it
           * covers; a bracket drawn with those weights is the bracket of a
           * point spread uniformly over that interval, (N_before + u6) eps/(rho V). */
          double vol = ldexp(h * h * h, -3 * lev);
          double nb = (double)before;
          if (p->flags & ORC_FLAG_EXACT_BW) nb += u[6];
          double pw = nb * eps / (p->rho[cell] * vol);
          const double *E = t->E + (int64_t)sp * K;
          int kb;
          if (pw < E[0]) { kb = 0; add_u64(&cnt[ORC_CNT_TCLAMP_LO], 1, thr); }
          else {
            int a = 0, b = K - 1;          /* E[a] <= pw, find largest such a */
            if (E[K - 1] <= pw) a = K - 1;
            else while (b - a > 1) { int m = (a + b) / 2; if (E[m] <= pw) a = m; else b = m; }
            kb = a;
            if (kb > K - 2) { kb = K - 2; add_u64(&cnt[ORC_CNT_TCLAMP_HI], 1, thr); }
          }
          j = cdf_search(t->R + ((int64_t)sp * (K - 1) + kb) * nl, nl, u[4]);
        } else {
          const int64_t slot = (int64_t)pah_slot[sp] * p->n_cells + cell;
          const double *row = p->pah_rows + (p->pah_row_map ? (int64_t)p->pah_row_map[slot] : slot) * nl;
          j = cdf_search(row, nl, u[4]);
          add_u64(&cnt[ORC_CNT_PAH_ABS], 1, thr);
        }
        iso_dir(2.0 * u[5] - 1.0, 2.0 * PI * u[2], d);
        tau = -log(u[3]);
        peel_tally(p, t, o, x, cell, lev, lo, j, NULL, thr);
        rec(o, k, ORC_EV_ABSORB, cell, j, x, d, tau);
      }
      continue;
    }
    /* cross the face to the neighbour */
    if (alpha > 0.0) tau -= alpha * tex;
    if ((p->flags & ORC_FLAG_TALLY_J) && dusty) {
      add_u64(&o->jq[(int64_t)j * p->n_cells + cell], (uint64_t)rint(tex * qscale), thr);
      add_u64(&cnt[ORC_CNT_JSEG], 1, thr);
    }
    add_u64(&cnt[ORC_CNT_CROSSINGS], 1, thr);
    if (tex == 0.0) add_u64(&cnt[ORC_CNT_ZERO_CROSS], 1, thr);
    for (int a = 0; a < 3; ++a) x[a] += tex * d[a];
    int64_t span = (int64_t)1 << (L - lev);
    x[ax] = (double)(d[ax] > 0.0 ? lo[ax] + span : lo[ax]) / (double)nf;
    int64_t G[3];
    for (int a = 0; a < 3; ++a) {
      if (a == ax) G[a] = d[a] > 0.0 ? lo[a] + span : lo[a] - 1;
      else {
        int64_t f = (int64_t)floor(x[a] * (double)nf);
        if (f < lo[a]) f = lo[a];
        if (f > lo[a] + span - 1) f = lo[a] + span - 1;
        G[a] = f;
      }
    }
    cell = orc_locate(p, G, &lev, lo);
    if (cell < 0) {
      add_u64(&cnt[ORC_CNT_ESCAPED], 1, thr);
      escape_tally(p, o, d, j, thr);
      image_tally(p, o, x, d, j, thr);
      rec(o, k, ORC_EV_ESCAPE, -1, j, x, d, tau);
      return;
    }
    rec(o, k, ORC_EV_CROSS, cell, j, x, d, tau);
  }
}

int orc_transport(const orc_problem *p, const orc_tables *t, uint64_t first_id, uint64_t n,
                  orc_out *o) {
  int32_t pah_slot[256];
  int np = 0;
  if (p->S > 256) return -1;
  for (int s = 0; s < p->S; ++s) pah_slot[s] = p->kind[s] == 1 ? np++ : -1;
  if (np > 0 && !p->pah_rows) return -2;
  if (o->trace) for (uint64_t k = 0; k < n; ++k) o->trace_len[k] = 0;
  if (p->n_threads <= 1) {
    for (uint64_t k = 0; k < n; ++k) run_packet(p, t, first_id + k, k, o, pah_slot, 0);
  } else {
#ifdef _OPENMP
    #pragma omp parallel for schedule(dynamic, 64) num_threads(p->n_threads)
    for (int64_t k = 0; k < (int64_t)n; ++k) run_packet(p, t, first_id + (uint64_t)k, (uint64_t)k, o, pah_slot, 1);
#else
    for (uint64_t k = 0; k < n; ++k) run_packet(p, t, first_id + k, k, o, pah_slot, 1);
#endif
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* temperatures and mean intensity                                            */
/* ------------------------------------------------------------------------ */
static double emission(const orc_problem *p, const orc_tables *t, int s, double T) {
  double e = 0.0;
  for (int j = 0; j < p->nl; ++j) e += p->kabs[s * p->nl + j] * orc_planck_nu(t->nu[j], T) * t->dnu[j];
  return 4.0 * PI * e;
}

/* volume (cm^3) of every leaf, from its depth in the tree */
static void leaf_volumes_rec(const orc_problem *p, int32_t e, int lev, double *vol) {
  if (e >= 0) { vol[e] = ldexp(p->base_size * p->base_size * p->base_size, -3 * lev); return; }
  for (int o = 0; o < 8; ++o) leaf_volumes_rec(p, p->nodes[(int64_t)(-e - 1) * 8 + o], lev + 1, vol);
}

static double *leaf_volumes(const orc_problem *p) {
  double *vol = (double *)malloc(sizeof(double) * (size_t)p->n_cells);
  int64_t nbase = (int64_t)p->nb * p->nb * p->nb;
  for (int64_t b = 0; b < nbase; ++b) leaf_volumes_rec(p, p->base_map[b], 0, vol);
  return vol;
}

/* Equilibrium temperature of every (cell, equilibrium species): the T at which
 * the grains give out what they absorbed, N_abs eps = rho V E_s(T), found by
 * bisection on [T_lo, T_hi]; T_lo when nothing was absorbed, clamped at the
 * ends.  PAH species get 0. */
void orc_temperatures(const orc_problem *p, const orc_tables *t, const uint64_t *nabs, double *T_out) {
  const double eps = p->lum / (double)p->n_total;
  double *vol = leaf_volumes(p);
  #pragma omp parallel for schedule(dynamic, 256) num_threads(p->n_threads > 0 ? p->n_threads : 1)
  for (int64_t c = 0; c < p->n_cells; ++c) {
    for (int s = 0; s < p->S; ++s) {
      double *T = &T_out[c * p->S + s];
      if (p->kind[s] != 0) { *T = 0.0; continue; }
      uint64_t N = nabs[c * p->S + s];
      if (N == 0 || p->rho[c] <= 0.0) { *T = p->T_lo; continue; }
      double pw = (double)N * eps / (p->rho[c] * vol[c]);
      double a = p->T_lo, b = p->T_hi;
      if (pw <= emission(p, t, s, a)) { *T = a; continue; }
      if (pw >= emission(p, t, s, b)) { *T = b; continue; }
      for (int it = 0; it < 200 && (b - a) > 1e-15 * b; ++it) {
        double m = 0.5 * (a + b);
        if (emission(p, t, s, m) <= pw) a = m; else b = m;
      }
      *T = 0.5 * (a + b);
    }
  }
  free(vol);
}

/* Path-length estimator of the mean intensity (Lucy 1999, the method the
 * packet scheme goes back to): J_nu = eps * sum(l) / (4 pi V dnu), with the
 * path sums held in fixed point (unit: finest cell side * 2^-16). */
void orc_mean_intensity(const orc_problem *p, const orc_tables *t, const uint64_t *jq, double *J_out) {
  const double eps = p->lum / (double)p->n_total;
  const double dq = p->base_size * ldexp(1.0, -(p->L + 16));   /* cm per unit */
  double *vol = leaf_volumes(p);
  for (int64_t c = 0; c < p->n_cells; ++c)
    for (int j = 0; j < p->nl; ++j)
      J_out[c * p->nl + j] = eps * dq * (double)jq[(int64_t)j * p->n_cells + c] / (4.0 * PI * vol[c] * t->dnu[j]);
  free(vol);
}

/* ------------------------------------------------------------------------ */
/* PAH: steady-state temperature distribution of transiently heated          */
/* molecules (Sec. 1, Sec. 4 and Fig. 3 of the paper).                       */
/*                                                                          */
/* States: M enthalpy bins with centres U_i = U(T_i).                        */
/* Heating (photon absorption; cross-section and field constant in each      */
/* wavelength bin, every photon of bin j carrying E_j = h nu_j):             */
/*   N_j = 4 pi C_j J_j dnu_j / (h nu_j) photons per second.                 */
/* A molecule in state i that absorbs one of them has enthalpy x = U_i + E_j;*/
/* the transition is shared between the two bin centres around x,            */
/* U_k <= x < U_{k+1}, with weights (U_{k+1} - x)/(U_{k+1} - U_k) on k and    */
/* (x - U_k)/(U_{k+1} - U_k) on k+1, so the mean enthalpy gain is exactly     */
/* E_j (the part left on k = i is no transition).  Jumps to or beyond the    */
/* top centre go to the top bin.  Hence sum_k A_{k,i} (U_k - U_i) equals the  */
/* absorbed power 4 pi sum_j C_j J_j dnu_j for every state whose jumps stay   */
/* below the top, and the steady state emits what it absorbs.                */
/* Cooling: continuous, to the next lower bin,                               */
/*   A_{i-1,i} = 4 pi sum_j C_j B_j(T_i) dnu_j / (U_i - U_{i-1}).             */
/* Steady state: the upward flux across the boundary below bin f equals the   */
/* downward flux P_f A_{f-1,f}, so with B_{f,i} = sum_{k>=f} A_{k,i}:        */
/*   P_f = sum_{i<f} B_{f,i} P_i / A_{f-1,f},   P_0 = 1, then normalised.     */
/* Outputs: 17 band powers sum_{i>=1} P_i 4 pi sum_j Cband_b(j) B_j(T_i) dnu_j */
/* and the continuum power per wavelength bin, per molecule (the ground bin   */
/* emits nothing, matching its lack of a downward transition).              */
/* ------------------------------------------------------------------------ */
void orc_pah_rates(int32_t M, const double *T, const double *U, int32_t nl,
                   const double *lam_um, const double *cabs, const double *J,
                   double *A_up, double *A_down) {
  double *nu = (double *)malloc(sizeof(double) * nl), *dnu = (double *)malloc(sizeof(double) * nl);
  orc_lambda_bins(nl, lam_um, nu, dnu);
  for (int64_t q = 0; q < (int64_t)M * M; ++q) A_up[q] = 0.0;
  for (int i = 0; i < M - 1; ++i) {
    for (int j = 0; j < nl; ++j) {
      const double E = H_PLANCK * nu[j];
      const double N = 4.0 * PI * cabs[j] * J[j] * dnu[j] / E;
      const double x = U[i] + E;
      if (x >= U[M - 1]) { A_up[(int64_t)(M - 1) * M + i] += N; continue; }
      int k = i;                                  /* U_k <= x < U_{k+1} */
      while (U[k + 1] <= x) ++k;
      const double span = U[k + 1] - U[k];
      if (k > i) A_up[(int64_t)k * M + i] += N * ((U[k + 1] - x) / span);
      A_up[(int64_t)(k + 1) * M + i] += N * ((x - U[k]) / span);
    }
  }
  A_down[0] = 0.0;
  for (int i = 1; i < M; ++i) {
    double pe = 0.0;
    for (int j = 0; j < nl; ++j) pe += cabs[j] * orc_planck_nu(nu[j], T[i]) * dnu[j];
    A_down[i] = 4.0 * PI * pe / (U[i] - U[i - 1]);
  }
  free(nu); free(dnu);
}

void orc_pah_solve(int32_t M, const double *T, const double *U, int32_t nl,
                   const double *lam_um, const double *cabs, const double *cband,
                   int32_t n_bands, const double *ccont, const double *J, int64_t n,
                   double *out, double *P_out, double *pabs_out, int32_t n_threads) {
  double *nu = (double *)malloc(sizeof(double) * nl), *dnu = (double *)malloc(sizeof(double) * nl);
  orc_lambda_bins(nl, lam_um, nu, dnu);
  const int n_out = n_bands + nl;
  /* per-bin emission of each output at each state temperature */
  double *em = (double *)malloc(sizeof(double) * (size_t)M * n_out);
  for (int i = 0; i < M; ++i) {
    for (int b = 0; b < n_bands; ++b) {
      double s = 0.0;
      for (int j = 0; j < nl; ++j) s += cband[(int64_t)b * nl + j] * orc_planck_nu(nu[j], T[i]) * dnu[j];
      em[(int64_t)i * n_out + b] = 4.0 * PI * s;
    }
    for (int j = 0; j < nl; ++j)
      em[(int64_t)i * n_out + n_bands + j] = 4.0 * PI * ccont[j] * orc_planck_nu(nu[j], T[i]) * dnu[j];
  }
  #pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int64_t c = 0; c < n; ++c) {
    const double *Jc = J + c * nl;
    double *A = (double *)malloc(sizeof(double) * (size_t)M * M);
    double *Ad = (double *)malloc(sizeof(double) * M);
    double *B = (double *)malloc(sizeof(double) * (size_t)M * M);
    double *P = (double *)malloc(sizeof(double) * M);
    orc_pah_rates(M, T, U, nl, lam_um, cabs, Jc, A, Ad);
    /* B_{f,i} = sum_{k >= f} A_{k,i}, summed from the top down */
    for (int i = 0; i < M; ++i) {
      double acc = 0.0;
      for (int f = M - 1; f > i; --f) { acc += A[(int64_t)f * M + i]; B[(int64_t)f * M + i] = acc; }
    }
    P[0] = 1.0;
    for (int f = 1; f < M; ++f) {
      double s = 0.0;
      for (int i = 0; i < f; ++i) s += B[(int64_t)f * M + i] * P[i];
      P[f] = s / Ad[f];
      /* keep the unnormalised P finite: rescale by an exact power of two */
      if (P[f] > 1e200) for (int i = 0; i <= f; ++i) P[i] = ldexp(P[i], -664);
    }
    double tot = 0.0;
    for (int i = 0; i < M; ++i) tot += P[i];
    for (int i = 0; i < M; ++i) P[i] /= tot;
    /* the ground bin has no lower state to cool to: it emits nothing */
    for (int q = 0; q < n_out; ++q) {
      double s = 0.0;
      for (int i = 1; i < M; ++i) s += P[i] * em[(int64_t)i * n_out + q];
      out[c * n_out + q] = s;
    }
    if (P_out) for (int i = 0; i < M; ++i) P_out[c * M + i] = P[i];
    if (pabs_out) {
      double pa = 0.0;
      for (int j = 0; j < nl; ++j) pa += cabs[j] * Jc[j] * dnu[j];
      pabs_out[c] = 4.0 * PI * pa;
    }
    free(A); free(Ad); free(B); free(P);
  }
  free(nu); free(dnu); free(em);
}

/* ------------------------------------------------------------------------ */
/* PAH re-emission rows: a packet absorbed by a PAH species leaves at a      */
/* wavelength drawn from the cell's PAH emission spectrum.  Per bin j:      */
/* continuum power cont_j plus every band's power F_b spread over the bins  */
/* in proportion to Cband_b(j) dnu_j (the band profile; the Planck factor   */
/* varies little across a band).  The row is the normalised running sum.    */
/* ------------------------------------------------------------------------ */
void orc_pah_rows(int32_t nl, int32_t n_bands, const double *lam_um, const double *cband,
                  const double *out, int64_t n, double *rows) {
  double *nu = (double *)malloc(sizeof(double) * nl), *dnu = (double *)malloc(sizeof(double) * nl);
  orc_lambda_bins(nl, lam_um, nu, dnu);
  double *w = (double *)malloc(sizeof(double) * (size_t)n_bands * nl);
  for (int b = 0; b < n_bands; ++b) {
    double tot = 0.0;
    for (int j = 0; j < nl; ++j) tot += cband[(int64_t)b * nl + j] * dnu[j];
    for (int j = 0; j < nl; ++j) w[(int64_t)b * nl + j] = tot > 0.0 ? cband[(int64_t)b * nl + j] * dnu[j] / tot : 0.0;
  }
  const int n_out = n_bands + nl;
  for (int64_t c = 0; c < n; ++c) {
    const double *o = out + c * n_out;
    double *r = rows + c * nl;
    double cum = 0.0;
    for (int j = 0; j < nl; ++j) {
      double e = o[n_bands + j];
      for (int b = 0; b < n_bands; ++b) e += o[b] * w[(int64_t)b * nl + j];
      cum += e;
      r[j] = cum;
    }
    for (int j = 0; j < nl; ++j) r[j] = cum > 0.0 ? r[j] / cum : 1.0;
    r[nl - 1] = 1.0;
  }
  free(nu); free(dnu); free(w);
}

/* ------------------------------------------------------------------------ */
/* Optically thin stellar field at every leaf centre, the starting field of */
/* the PAH iteration: J_nu,j = L w_j / (16 pi^2 r^2 dnu_j), w_j the source's */
/* share of bin j, r the distance star - centre, at least half the side.    */
/* ------------------------------------------------------------------------ */
static void leaf_centres_rec(const orc_problem *p, int32_t e, int lev, int64_t lo0, int64_t lo1,
                             int64_t lo2, double *cen, double *half) {
  const int64_t span = (int64_t)1 << (p->L - lev);
  if (e >= 0) {
    const double fine = p->base_size * ldexp(1.0, -p->L);
    cen[3 * e + 0] = p->box_min[0] + ((double)lo0 + 0.5 * (double)span) * fine;
    cen[3 * e + 1] = p->box_min[1] + ((double)lo1 + 0.5 * (double)span) * fine;
    cen[3 * e + 2] = p->box_min[2] + ((double)lo2 + 0.5 * (double)span) * fine;
    half[e] = 0.5 * (double)span * fine;
    return;
  }
  const int64_t h = span >> 1;
  for (int o = 0; o < 8; ++o)
    leaf_centres_rec(p, p->nodes[(int64_t)(-e - 1) * 8 + o], lev + 1, lo0 + (o & 1) * h,
                     lo1 + ((o >> 1) & 1) * h, lo2 + ((o >> 2) & 1) * h, cen, half);
}

void orc_thin_field(const orc_problem *p, const orc_tables *t, double *J_out) {
  double *cen = (double *)malloc(sizeof(double) * 3 * (size_t)p->n_cells);
  double *half = (double *)malloc(sizeof(double) * (size_t)p->n_cells);
  const int64_t nf = (int64_t)1 << p->L;
  for (int64_t b = 0; b < (int64_t)p->nb * p->nb * p->nb; ++b) {
    int64_t bx = b % p->nb, by = (b / p->nb) % p->nb, bz = b / ((int64_t)p->nb * p->nb);
    leaf_centres_rec(p, p->base_map[b], 0, bx * nf, by * nf, bz * nf, cen, half);
  }
  for (int64_t c = 0; c < p->n_cells; ++c) {
    double dx = cen[3 * c] - p->src_pos[0], dy = cen[3 * c + 1] - p->src_pos[1], dz = cen[3 * c + 2] - p->src_pos[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r < half[c]) r = half[c];
    for (int j = 0; j < p->nl; ++j) {
      double w = t->src_cdf[j] - (j > 0 ? t->src_cdf[j - 1] : 0.0);
      J_out[c * p->nl + j] = p->lum * w / (16.0 * PI * PI * r * r * t->dnu[j]);
    }
  }
  free(cen); free(half);
}
