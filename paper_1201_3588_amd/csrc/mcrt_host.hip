// C ABI of the transport engine: descriptor validation, error codes, launches
// on the caller's stream.  No exception crosses the boundary.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mcrt_internal.h"

using namespace mcrt;

namespace {

int32_t fail(mcrt_ctx* c, int32_t code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int32_t hip_fail(mcrt_ctx* c, hipError_t e, const char* where) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
  return fail(c, MCRT_E_HIP, buf);
}

const char* check_desc(const mcrt_desc* d) {
  if (!d) return "null descriptor";
  if (d->precision != MCRT_F32 && d->precision != MCRT_F64) return "precision must be MCRT_F32 or MCRT_F64";
  if (d->n_lambda < 2) return "n_lambda must be >= 2";
  if (d->n_species < 1 || d->n_species > 256) return "n_species must be in 1..256";
  if (d->nb < 1) return "nb must be >= 1";
  if (d->max_level < 0 || d->max_level > 10) return "max_level must be in 0..10";
  if ((int64_t)d->nb << d->max_level > (1 << 20)) return "nb * 2^max_level must be <= 2^20";
  if ((int64_t)d->nb * d->nb * d->nb > (int64_t)1 << 31) return "nb^3 too large";
  if (d->K < 2) return "K must be >= 2";
  if (d->n_cells < 1 || d->n_cells >= ((int64_t)1 << 31)) return "n_cells out of range";
  if (d->n_nodes < 0 || d->n_nodes >= ((int64_t)1 << 28)) return "n_nodes out of range";
  if (d->n_nodes > 0 && d->max_level < 1) return "nodes need max_level >= 1";
  if (!(d->base_size > 0.0) || !std::isfinite(d->base_size)) return "base_size must be > 0";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->box_min[a])) return "box_min must be finite";
  if (!(d->T_lo > 0.0) || !(d->T_hi > d->T_lo) || !std::isfinite(d->T_hi)) return "need 0 < T_lo < T_hi";
  if (d->n_theta < 1 || d->n_phi < 1) return "n_theta, n_phi must be >= 1";
  if (!d->lambda_um || !d->kabs || !d->ksca || !d->g || !d->kind || !d->base_map || !d->rho)
    return "null device array in descriptor";
  if (d->n_nodes > 0 && !d->nodes) return "nodes is null but n_nodes > 0";
  return nullptr;
}

}  // namespace

extern "C" {

int32_t mcrt_version(void) { return MCRT_VERSION; }

int32_t mcrt_tables_bytes(const mcrt_desc* desc, uint64_t* bytes) {
  if (check_desc(desc) || !bytes) return MCRT_E_INVALID;
  *bytes = make_layout(*desc).total;
  return MCRT_OK;
}

int32_t mcrt_ctx_create(const mcrt_desc* desc, mcrt_ctx** out) {
  if (!out) return MCRT_E_INVALID;
  *out = nullptr;
  if (check_desc(desc)) return MCRT_E_INVALID;
  mcrt_ctx* c = new (std::nothrow) mcrt_ctx();
  if (!c) return MCRT_E_INVALID;
  c->d = *desc;
  c->lay = make_layout(*desc);
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    c->device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      c->n_cu = ncu;
  }
  *out = c;
  return MCRT_OK;
}

void mcrt_ctx_destroy(mcrt_ctx* ctx) { delete ctx; }

const char* mcrt_last_error(const mcrt_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t mcrt_table_layout_get(const mcrt_ctx* ctx, mcrt_table_layout* out) {
  if (!ctx || !out) return MCRT_E_INVALID;
  const Layout& L = ctx->lay;
  *out = mcrt_table_layout{L.nu, L.dnu, L.src_cdf, L.kext, L.albedo, L.gpar, L.sp_cdf, L.Tk, L.E,
                           L.R, L.Bt, L.Wt, L.xk, L.kext32, L.g32, L.rho_h32, L.level, L.leaf_lo, L.binfo, L.pah_slot, L.scratch,
                           L.total};
  return MCRT_OK;
}

int32_t mcrt_build_tables(mcrt_ctx* ctx, const mcrt_source* src, void* tables, uint64_t tables_bytes,
                          hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!src || !tables) return fail(ctx, MCRT_E_INVALID, "null source or tables");
  if (tables_bytes < ctx->lay.total) return fail(ctx, MCRT_E_CAPACITY, "tables buffer too small");
  if (!(src->teff > 0.0) || !std::isfinite(src->teff)) return fail(ctx, MCRT_E_NUMERIC, "teff must be > 0");
  if (!(src->lum > 0.0) || !std::isfinite(src->lum)) return fail(ctx, MCRT_E_NUMERIC, "lum must be > 0");
  if (src->beam_on) {
    const double n = std::sqrt(src->beam[0] * src->beam[0] + src->beam[1] * src->beam[1] +
                               src->beam[2] * src->beam[2]);
    if (!(std::fabs(n - 1.0) < 1e-6)) return fail(ctx, MCRT_E_NUMERIC, "beam must be a unit vector");
  }
  ctx->tables = static_cast<unsigned char*>(tables);
  ctx->src = *src;
  ctx->tables_built = false;
  hipError_t e = launch_checks(ctx, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "input check launch");
  unsigned long long bad = 0;
  std::vector<int32_t> kind(ctx->d.n_species);
  e = hipMemcpyAsync(&bad, ctx->tables + ctx->lay.scratch + offsetof(RunScratch, bad_input),
                     sizeof bad, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(kind.data(), ctx->d.kind, sizeof(int32_t) * kind.size(),
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "input check");
  if (bad & 16ull) return fail(ctx, MCRT_E_INVALID, "grid structure invalid (range, order or depth)");
  ctx->n_pah = 0;
  for (int32_t k : kind) {
    if (k != 0 && k != 1) return fail(ctx, MCRT_E_INVALID, "species kind must be 0 or 1");
    ctx->n_pah += k == 1;
  }
  if (bad) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "input values invalid (flags 0x%llx: 1 rho, 2 opacity, 4 lambda, 8 g)", bad);
    return fail(ctx, MCRT_E_NUMERIC, buf);
  }
  e = launch_build_tables(ctx, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "table build launch");
  ctx->tables_built = true;
  return MCRT_OK;
}

int32_t mcrt_set_observers(mcrt_ctx* ctx, const mcrt_observers* obs) {
  if (!ctx) return MCRT_E_INVALID;
  if (!obs) return fail(ctx, MCRT_E_INVALID, "null observers");
  if (obs->n_obs == 0) {
    ctx->img = ImgP{};
    return MCRT_OK;
  }
  if (obs->n_obs < 0 || obs->n_obs > MCRT_MAX_OBSERVERS) return fail(ctx, MCRT_E_INVALID, "n_obs must be in 0..8");
  if (obs->npix < 1 || obs->npix > 4096) return fail(ctx, MCRT_E_INVALID, "npix must be in 1..4096");
  if (obs->n_img_lambda < 1 || obs->n_img_lambda > MCRT_MAX_IMAGE_BINS)
    return fail(ctx, MCRT_E_INVALID, "n_img_lambda must be in 1..8");
  if (!(obs->half_width > 0.0) || !std::isfinite(obs->half_width))
    return fail(ctx, MCRT_E_INVALID, "half_width must be positive and finite");
  if (!(obs->cos_cone > 0.0 && obs->cos_cone <= 1.0)) return fail(ctx, MCRT_E_INVALID, "cos_cone must be in (0, 1]");
  ImgP I{};
  I.n_obs = obs->n_obs;
  I.npix = obs->npix;
  I.n_l = obs->n_img_lambda;
  for (int q = 0; q < I.n_l; ++q) {
    const int jb = obs->img_lambda[q];
    if (jb < 0 || jb >= ctx->d.n_lambda) return fail(ctx, MCRT_E_INVALID, "imaged bin out of range");
    for (int r = 0; r < q; ++r)
      if (I.lsel[r] == jb) return fail(ctx, MCRT_E_INVALID, "imaged bins must be distinct");
    I.lsel[q] = jb;
  }
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(obs->center[a])) return fail(ctx, MCRT_E_INVALID, "center not finite");
    I.off[a] = ctx->d.box_min[a] - obs->center[a];
  }
  for (int o = 0; o < I.n_obs; ++o) {
    const double* m = obs->dir[o];
    const double len = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    if (!(len > 0.0) || !std::isfinite(len)) return fail(ctx, MCRT_E_INVALID, "observer direction zero or not finite");
    double* n = I.n[o];
    for (int a = 0; a < 3; ++a) n[a] = m[a] / len;
    double* e1 = I.e1[o];
    double* e2 = I.e2[o];
    const double r = std::sqrt(n[0] * n[0] + n[1] * n[1]);   // |z x n|
    if (r > 1e-12) { e1[0] = -n[1] / r; e1[1] = n[0] / r; e1[2] = 0.0; }
    else { e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0; }
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];
  }
  I.h = ctx->d.base_size;
  I.w = obs->half_width;
  I.cos_cone = obs->cos_cone;
  ctx->img = I;
  return MCRT_OK;
}

int32_t mcrt_read_counters_sync(const mcrt_tallies* t, uint64_t* host_out, hipStream_t stream) {
  if (!t || !t->counters || !host_out) return MCRT_E_INVALID;
  hipError_t e = hipMemcpyAsync(host_out, t->counters, sizeof(uint64_t) * MCRT_N_COUNTERS,
                                hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

int32_t mcrt_run(mcrt_ctx* ctx, uint64_t first_id, uint64_t n_packets, const mcrt_run_opts* opts,
                 const mcrt_tallies* tallies, hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!ctx->tables_built) return fail(ctx, MCRT_E_STATE, "mcrt_run before mcrt_build_tables");
  if (!opts || !tallies) return fail(ctx, MCRT_E_INVALID, "null opts or tallies");
  if (!tallies->nabs || !tallies->sed || !tallies->counters)
    return fail(ctx, MCRT_E_INVALID, "null tally array");
  if ((opts->flags & MCRT_FLAG_TALLY_J) && !tallies->jq)
    return fail(ctx, MCRT_E_INVALID, "TALLY_J needs tallies->jq");
  if ((opts->flags & MCRT_FLAG_FROZEN_T) && !opts->frozen_nabs)
    return fail(ctx, MCRT_E_INVALID, "FROZEN_T needs frozen_nabs");
  if (opts->flags & ~63) return fail(ctx, MCRT_E_INVALID, "unknown flag bits");
  if ((opts->flags & MCRT_FLAG_PEEL_SED) && !(opts->flags & MCRT_FLAG_PEEL))
    return fail(ctx, MCRT_E_INVALID, "PEEL_SED needs PEEL");
  if (opts->flags & MCRT_FLAG_PEEL) {
    if (ctx->img.n_obs == 0) return fail(ctx, MCRT_E_INVALID, "PEEL needs observers");
    if (!tallies->peel) return fail(ctx, MCRT_E_INVALID, "PEEL needs tallies->peel");
    if ((opts->flags & MCRT_FLAG_PEEL_SED) && !tallies->peel_sed)
      return fail(ctx, MCRT_E_INVALID, "PEEL_SED needs tallies->peel_sed");
    if (!opts->peel_queue || opts->peel_capacity < 1)
      return fail(ctx, MCRT_E_INVALID, "PEEL needs peel_queue and peel_capacity >= 1");
  }
  if (opts->n_total == 0) return fail(ctx, MCRT_E_INVALID, "n_total must be > 0");
  if (opts->trace && (!opts->trace_len || opts->trace_cap < 1))
    return fail(ctx, MCRT_E_INVALID, "trace needs trace_len and trace_cap >= 1");
  if (first_id + n_packets < first_id) return fail(ctx, MCRT_E_INVALID, "packet id range overflows");
  if (ctx->n_pah > 0 && !opts->pah_rows && !(opts->flags & MCRT_FLAG_KILL_ON_ABSORB))
    return fail(ctx, MCRT_E_INVALID, "PAH species need pah_rows");
  if (ctx->img.n_obs > 0 && !tallies->image)
    return fail(ctx, MCRT_E_INVALID, "observers are set: tallies->image needed");
  if (opts->jrec_ws) {
    if (!(opts->flags & MCRT_FLAG_TALLY_J) || !tallies->jq)
      return fail(ctx, MCRT_E_INVALID, "jrec_ws needs TALLY_J and tallies->jq");
    uint64_t need = 0;
    const int32_t rc = mcrt_jrec_ws_bytes(ctx, opts->jrec_capacity, &need);
    if (rc != MCRT_OK) return fail(ctx, rc, "jrec_capacity out of range or grid unsupported for the deferred tally");
  }
  if (n_packets == 0) return MCRT_OK;
  const hipError_t e = launch_transport(ctx, first_id, n_packets, *opts, *tallies, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "transport launch");
  return MCRT_OK;
}

int32_t mcrt_temperatures(mcrt_ctx* ctx, const uint64_t* nabs, uint64_t n_total, double* T_out,
                          hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!ctx->tables_built) return fail(ctx, MCRT_E_STATE, "temperatures before mcrt_build_tables");
  if (!nabs || !T_out || n_total == 0) return fail(ctx, MCRT_E_INVALID, "null array or n_total == 0");
  const hipError_t e = launch_temperatures(ctx, nabs, n_total, T_out, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "temperature launch");
  return MCRT_OK;
}

int32_t mcrt_thin_field(mcrt_ctx* ctx, float* J_out, hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!ctx->tables_built) return fail(ctx, MCRT_E_STATE, "thin field before mcrt_build_tables");
  if (!J_out) return fail(ctx, MCRT_E_INVALID, "null J_out");
  const hipError_t e = launch_thin_field(ctx, J_out, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "thin field launch");
  return MCRT_OK;
}

int32_t mcrt_cell_mass(mcrt_ctx* ctx, double* mass_out, hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!ctx->tables_built) return fail(ctx, MCRT_E_STATE, "cell mass before mcrt_build_tables");
  if (!mass_out) return fail(ctx, MCRT_E_INVALID, "null mass_out");
  const hipError_t e = launch_cell_mass(ctx, mass_out, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cell mass launch");
  return MCRT_OK;
}

int32_t mcrt_mean_intensity(mcrt_ctx* ctx, const uint64_t* jq, uint64_t n_total, float* J_out,
                            hipStream_t stream) {
  if (!ctx) return MCRT_E_INVALID;
  if (!ctx->tables_built) return fail(ctx, MCRT_E_STATE, "mean intensity before mcrt_build_tables");
  if (!jq || !J_out || n_total == 0) return fail(ctx, MCRT_E_INVALID, "null array or n_total == 0");
  const hipError_t e = launch_mean_intensity(ctx, jq, n_total, J_out, stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "mean intensity launch");
  return MCRT_OK;
}

}  // extern "C"
