/* Drives every entry point of the CPU oracle on a tiny nested grid, for runs
 * under the host sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer,
 * ThreadSanitizer for the threaded transport).  Exit status 0 when every
 * call returned normally and the packet bookkeeping balances. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/mcrt_oracle.h"

#define NL 8
#define NSP 2

static double *dz(size_t n) { return (double *)calloc(n, sizeof(double)); }

int main(int argc, char **argv) {
  const int threads = argc > 1 ? atoi(argv[1]) : 1;
  /* 2^3 base cubes of 1 cm, the first refined once (8 leaves): 15 leaves */
  int32_t base_map[8], nodes[8];
  base_map[0] = -1;
  for (int o = 0; o < 8; ++o) nodes[o] = o;
  for (int b = 1; b < 8; ++b) base_map[b] = 8 + (b - 1);
  const int64_t n_cells = 15;
  double rho[15], lam[NL], kabs[NSP * NL], ksca[NSP * NL], g[NL];
  int32_t kind[NSP] = {0, 0};
  for (int c = 0; c < n_cells; ++c) rho[c] = c == 3 ? 0.0 : 1.0 + 0.1 * c;
  for (int j = 0; j < NL; ++j) {
    lam[j] = 0.1 * pow(10.0, 4.0 * j / (NL - 1));
    g[j] = 0.3;
    for (int s = 0; s < NSP; ++s) {
      kabs[s * NL + j] = (0.3 + 0.2 * s) / (1.0 + lam[j]);
      ksca[s * NL + j] = 0.2 / (1.0 + lam[j] * lam[j]);
    }
  }
  orc_problem p;
  memset(&p, 0, sizeof p);
  p.nl = NL; p.S = NSP; p.lam_um = lam; p.kabs = kabs; p.ksca = ksca; p.g = g; p.kind = kind;
  p.nb = 2; p.L = 1; p.n_cells = n_cells; p.n_nodes = 1;
  p.box_min[0] = p.box_min[1] = p.box_min[2] = 0.0; p.base_size = 1.0;
  p.base_map = base_map; p.nodes = nodes; p.rho = rho;
  p.src_pos[0] = 0.7; p.src_pos[1] = 0.9; p.src_pos[2] = 1.0;
  p.lum = 1.0; p.teff = 5000.0;
  p.K = 64; p.T_lo = 3.0; p.T_hi = 3000.0;
  p.n_total = 2000; p.seed = 11; p.max_events = 500;
  p.n_theta = 4; p.n_phi = 2; p.flags = 1; p.n_threads = threads;
  p.n_obs = 2; p.npix = 5; p.n_img_lambda = 2; p.img_lambda[0] = 2; p.img_lambda[1] = 3;
  p.img_center[0] = p.img_center[1] = p.img_center[2] = 1.0;
  p.img_half_width = 2.0; p.img_cos_cone = 0.7;
  p.obs_dir[0][2] = 1.0; p.obs_dir[1][0] = 1.0; p.obs_dir[1][1] = 1.0;

  orc_tables t;
  t.nu = dz(NL); t.dnu = dz(NL); t.src_cdf = dz(NL); t.kext = dz(NL); t.albedo = dz(NL);
  t.sp_cdf = dz(NL * NSP); t.Tk = dz(p.K); t.E = dz(NSP * p.K); t.R = dz((size_t)NSP * (p.K - 1) * NL);
  orc_build_tables(&p, &t);

  orc_out o;
  memset(&o, 0, sizeof o);
  o.nabs = (uint64_t *)calloc(n_cells * NSP, 8);
  o.sed = (uint64_t *)calloc(p.n_theta * p.n_phi * NL, 8);
  o.jq = (uint64_t *)calloc(NL * n_cells, 8);
  o.counters = (uint64_t *)calloc(16, 8);
  o.image = (uint64_t *)calloc(p.n_obs * p.n_img_lambda * p.npix * p.npix, 8);
  if (threads == 1) {
    o.trace_cap = 64;
    o.trace = (orc_trace_rec *)calloc(64 * 16, sizeof(orc_trace_rec));
    o.trace_len = (int32_t *)calloc(16, 4);
    if (orc_transport(&p, &t, 0, 16, &o) != 0) return 2;
    free(o.trace); free(o.trace_len);
    o.trace = NULL; o.trace_len = NULL; o.trace_cap = 0;
  } else if (orc_transport(&p, &t, 0, 16, &o) != 0) {
    return 2;
  }
  if (orc_transport(&p, &t, 16, p.n_total - 16, &o) != 0) return 3;
  const uint64_t *c = o.counters;
  if (c[0] != p.n_total || c[0] != c[1] + c[2] + c[3]) return 4;

  double *T = dz(n_cells * NSP), *J = dz(n_cells * NL), *Jt = dz(n_cells * NL);
  orc_temperatures(&p, &t, o.nabs, T);
  orc_mean_intensity(&p, &t, o.jq, J);
  orc_thin_field(&p, &t, Jt);
  for (int64_t q = 0; q < n_cells * NSP; ++q) if (!isfinite(T[q])) return 5;

  /* PAH: a 30-state toy molecule on the same bins */
  enum { M = 30, NB = 3 };
  double Tp[M], Up[M], cab[NL], cbd[NB * NL], ccn[NL];
  for (int i = 0; i < M; ++i) { Tp[i] = 3.0 * pow(1000.0, (double)i / (M - 1)); Up[i] = 1e-16 * pow(Tp[i], 1.5); }
  for (int j = 0; j < NL; ++j) {
    ccn[j] = 1e-18 / (1.0 + lam[j]);
    cab[j] = ccn[j];
    for (int b = 0; b < NB; ++b) { cbd[b * NL + j] = 1e-20 * (b + 1) / (1.0 + fabs(lam[j] - 10.0 * (b + 1))); cab[j] += cbd[b * NL + j]; }
  }
  double *A = dz(M * M), *Ad = dz(M), *out = dz(2 * (NB + NL)), *P = dz(2 * M), *pabs = dz(2), *rows = dz(2 * NL);
  orc_pah_rates(M, Tp, Up, NL, lam, cab, J, A, Ad);
  orc_pah_solve(M, Tp, Up, NL, lam, cab, cbd, NB, ccn, J, 2, out, P, pabs, threads);
  orc_pah_rows(NL, NB, lam, cbd, out, 2, rows);
  for (int k = 0; k < 2 * M; ++k) if (!isfinite(P[k])) return 6;
  printf("ok %llu %llu %llu\n", (unsigned long long)c[0], (unsigned long long)c[5], (unsigned long long)c[6]);
  return 0;
}
