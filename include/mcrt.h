/*
 * mcrt.h -- C ABI of the MI355X Monte Carlo dust radiative-transfer engine.
 *
 * Method (Siebenmorgen, Heymann & Kruegel, "PAH in vectorized three
 * dimensional Monte Carlo dust radiative transfer models", Sec. 2): a point
 * star emits photon packets of constant energy eps = L / N_total; each packet
 * flies cell by cell through a grid of base cubes and subcubes, interacting
 * where the extinction optical depth along its path reaches a sampled value;
 * a scattering changes only its direction (Henyey-Greenstein phase function);
 * an absorption adds eps to the cell and re-emits the packet isotropically
 * from the same spot at a frequency drawn from the temperature of the cell
 * *before* the absorption (the form without the Bjorkman & Wood correction,
 * which lets packets fly in parallel).
 *
 * Conventions for every entry point:
 *  - All arrays named "device" are caller-owned device memory (e.g. torch
 *    tensors); the library never allocates device memory (its only device
 *    memory of its own is the 1 KiB static array of mcrt_image_psf_static)
 *    and never frees caller memory.  Host structs are copied at the call.
 *  - Every launch is asynchronous on the given stream; results are visible
 *    after the stream is synchronised.  Only functions ending in _sync block.
 *  - Return value: MCRT_OK or a negative MCRT_E_* code; the message of the
 *    last error of a context is returned by mcrt_last_error.  No C++
 *    exception crosses the boundary.  Kernel faults surface at the next
 *    synchronising call as MCRT_E_HIP.
 *  - A context holds non-owning pointers to the descriptor's device arrays:
 *    they must outlive it.  Calls on one context must not overlap in time
 *    (they share the run scratch held in the tables buffer).
 */
#ifndef MCRT_H
#define MCRT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_VERSION 104

#define MCRT_OK 0
#define MCRT_E_INVALID (-1)     /* null pointer, bad size or range */
#define MCRT_E_STATE (-2)       /* wrong call order (e.g. run before tables) */
#define MCRT_E_HIP (-3)         /* HIP runtime error; message carries the code */
#define MCRT_E_CAPACITY (-4)    /* caller buffer too small */
#define MCRT_E_NUMERIC (-5)     /* NaN or negative input values */
#define MCRT_E_UNSUPPORTED (-6)

#define MCRT_F32 0              /* transport geometry in FP32 */
#define MCRT_F64 1              /* transport geometry in FP64 */

#define MCRT_FLAG_TALLY_J 1         /* path-length mean-intensity tally */
#define MCRT_FLAG_FROZEN_T 2        /* temperature bracket from frozen_nabs */
#define MCRT_FLAG_KILL_ON_ABSORB 4  /* test mode: absorption ends the packet */
/* Re-emission from the Bjorkman & Wood (2001) difference spectrum
 * kabs [B(T_after) - B(T_before)] of the absorption's own temperature rise
 * (the corrected law the paper's method drops, Sec. 2) instead of the bracket
 * holding T_before: the bracket is looked up at (N_before + u) eps / (rho V),
 * u the seventh uniform of the event, so the rows between the two temperatures
 * are drawn in proportion to the energy each covers. */
#define MCRT_FLAG_EXACT_BW 8
/* Next-event (peel-off) images for the observers; see mcrt_run_opts.peel_queue. */
#define MCRT_FLAG_PEEL 16
/* With MCRT_FLAG_PEEL: also each observer's next-event SED over every bin
 * (tallies->peel_sed); every emission and scattering is queued, not only
 * those in imaged bins. */
#define MCRT_FLAG_PEEL_SED 32

/* counter slots of mcrt_tallies.counters */
#define MCRT_CNT_LAUNCHED 0
#define MCRT_CNT_ESCAPED 1
#define MCRT_CNT_KILLED 2        /* hit the per-packet event cap */
#define MCRT_CNT_TERMINATED 3    /* ended by KILL_ON_ABSORB */
#define MCRT_CNT_SCATTERS 4
#define MCRT_CNT_ABSORPTIONS 5
#define MCRT_CNT_CROSSINGS 6     /* segments ending on a cell face */
#define MCRT_CNT_TCLAMP_LO 7     /* absorbed energy below E(T_lo) */
#define MCRT_CNT_TCLAMP_HI 8     /* absorbed energy at or above E(T_{K-2}) bracket */
#define MCRT_CNT_PAH_ABS 9
#define MCRT_CNT_ZERO_CROSS 10   /* zero-length face crossings (ties) */
#define MCRT_CNT_JSEG 11         /* segments added to the path-length tally */
#define MCRT_CNT_PEEL 12         /* events queued for the next-event images */
#define MCRT_CNT_PEEL_DROPPED 13 /* of those, not stored: peel_queue full */
#define MCRT_N_COUNTERS 16

typedef struct mcrt_ctx mcrt_ctx;

/* Problem description (paper Sec. 1 dust model, Sec. 2 grid).
 * Wavelength bins: centres lambda_um[j], edges at geometric midpoints,
 * cross-sections constant in a bin.  Opacities are cm^2 per gram of the dust
 * mixture (species mass fractions folded in); every species follows the same
 * density law rho (g cm^-3) per cell.  Grid: nb^3 base cubes of side
 * base_size (cm) from box_min; base_map[ix + nb*(iy + nb*iz)] is a leaf id
 * (>= 0) or -(node+1); nodes[8*node + o] for octant o = bx | by<<1 | bz<<2
 * uses the same encoding; leaves are max_level deep at most. */
typedef struct {
  int32_t precision;           /* MCRT_F32 or MCRT_F64 */
  int32_t n_lambda;            /* >= 2 */
  int32_t n_species;           /* 1..256 */
  int32_t nb;                  /* base cubes per axis */
  int32_t max_level;           /* 0..10, nb * 2^max_level <= 2^20 */
  int32_t K;                   /* temperature grid points, >= 2 */
  int64_t n_cells;             /* leaves */
  int64_t n_nodes;             /* interior nodes */
  double box_min[3];           /* cm */
  double base_size;            /* cm */
  double T_lo, T_hi;           /* temperature grid, log spaced, K */
  int32_t n_theta, n_phi;      /* escape-direction bins (equal cos, equal phi) */
  const double *lambda_um;     /* device [n_lambda], increasing */
  const double *kabs;          /* device [n_species * n_lambda] */
  const double *ksca;          /* device [n_species * n_lambda] */
  const double *g;             /* device [n_lambda] HG asymmetry */
  const int32_t *kind;         /* device [n_species]: 0 equilibrium, 1 PAH */
  const int32_t *base_map;     /* device [nb^3] */
  const int32_t *nodes;        /* device [8 * n_nodes] (may be NULL if 0) */
  const double *rho;           /* device [n_cells] */
} mcrt_desc;

/* Point source (paper Sec. 2: the star).  Blackbody of teff integrated over
 * the bins; isotropic unless beam_on (pencil beam along beam[], unit). */
typedef struct {
  double pos[3];               /* cm */
  double lum;                  /* erg s^-1 */
  double teff;                 /* K */
  double beam[3];
  int32_t beam_on;
} mcrt_source;

/* Integer tallies, device, accumulated (+=) by every run. */
typedef struct {
  uint64_t *nabs;              /* [n_cells * n_species] absorbed packets */
  uint64_t *sed;               /* [n_theta * n_phi * n_lambda] escaped packets */
  uint64_t *jq;                /* [n_lambda * n_cells] path sums, unit
                                  base_size * 2^-(max_level+16) cm; NULL if
                                  TALLY_J is off */
  uint64_t *counters;          /* [MCRT_N_COUNTERS] */
  uint64_t *image;             /* [n_obs][n_img_lambda][npix][npix] escaped
                                  packets per pixel (mcrt_observers); NULL
                                  when no observers are set */
  uint64_t *peel;              /* [n_obs][n_img_lambda][npix][npix] next-event
                                  weights in units of 2^-24 (MCRT_FLAG_PEEL);
                                  NULL when the flag is off */
  uint64_t *peel_sed;          /* [n_obs][n_lambda] next-event SED: the same
                                  weights of every event in bin j, wherever it
                                  projects (MCRT_FLAG_PEEL_SED); NULL when off */
} mcrt_tallies;

/* Escape images (paper Sec. 2, Fig. 2: the model seen from chosen
 * directions).  Observer o looks back along dir[o].  A packet that leaves the
 * grid in direction d with d . dir[o] >= cos_cone, in one of the imaged bins
 * img_lambda[l], is placed where its ray, extended backwards from the exit
 * point, crosses the image plane through `center` perpendicular to dir[o].
 * The plane's axes are e1 = (z x n)/|z x n| (the x axis when n is along z)
 * and e2 = n x e1 (n = dir[o] normalised); plane coordinates (a, b) map to
 * pixel (floor((a + w) / (2 w) npix), floor((b + w) / (2 w) npix)),
 * w = half_width, counted in image[o][l][py][px] when both lie in
 * [0, npix).  Direct starlight from a star at `center` lands in the centre. */
#define MCRT_MAX_OBSERVERS 8
#define MCRT_MAX_IMAGE_BINS 8
typedef struct {
  int32_t n_obs;               /* 0..8; 0 turns the images off */
  int32_t npix;                /* pixels per image side, 1..4096 */
  int32_t n_img_lambda;        /* 1..8 */
  int32_t img_lambda[MCRT_MAX_IMAGE_BINS];  /* distinct bins in [0, n_lambda) */
  int32_t pad;
  double center[3];            /* cm */
  double half_width;           /* cm, > 0 */
  double cos_cone;             /* (0, 1] */
  double dir[MCRT_MAX_OBSERVERS][3];        /* non-zero; normalised here */
} mcrt_observers;

/* Next-event (peel-off) images, MCRT_FLAG_PEEL (paper Sec. 4 and Fig. 2: the
 * disk imaged at 11.3 and 10 um).  At every emission of a packet in an imaged
 * bin (the star's, unless it is a pencil beam, and each re-emission after an
 * absorption) and every scattering in an imaged bin, each observer receives
 * the chance per unit solid angle that the packet leaves towards it, times
 * 4 pi: 1 for isotropic emission, the Henyey-Greenstein function
 * (1 - g^2) / (1 + g^2 - 2 g mu)^(3/2) for a scattering (mu: cosine between
 * the arriving direction and the line of sight; 1 when |g| < 1e-5), times
 * exp(-tau) of the path from the event to the edge of the grid along the
 * line of sight, at the pixel of the event's projection on the image plane
 * (the escape images' axes and pixels).  Each weight w is added as
 * round-to-nearest(2^24 w) to tallies->peel; a pixel's flux at distance D is
 * eps / (4 pi D^2) 2^-24 times its sum (erg s^-1 cm^-2 in its bin).  With
 * MCRT_FLAG_PEEL_SED the same rounded weight of every event, in any bin, is
 * also added to tallies->peel_sed[o][j] (the observer's SED, paper Sec. 2 and
 * Fig. 1: the flux towards that direction per bin, same scale).  The
 * transport stores one MCRT_PEEL_REC_BYTES record per such event in
 * opts->peel_queue (device, caller-owned, peel_capacity records); a second
 * kernel on the same stream then marches every record's lines of sight.
 * Events beyond the capacity are counted in MCRT_CNT_PEEL_DROPPED and are
 * missing from the images: run smaller id ranges.  A source outside the grid
 * adds no direct light. */
#define MCRT_PEEL_REC_BYTES 64
#define MCRT_PEEL_UNIT 16777216.0

/* Per-packet event trace (debug/test only). */
typedef struct {
  int32_t type, cell, j, pad;  /* type: 0 launch 1 cross 2 scatter 3 absorb 4 escape 5 killed */
  double x[3], d[3], tau;      /* x in base-cube units */
} mcrt_trace_rec;

typedef struct {
  uint64_t n_total;            /* packets of the whole pass: eps = lum / n_total */
  uint64_t seed;               /* Philox key */
  uint64_t max_events;         /* interactions per packet before it is killed */
  int32_t flags;               /* MCRT_FLAG_* */
  int32_t grid_blocks;         /* 0 = automatic */
  const uint64_t *frozen_nabs; /* device [n_cells * n_species] for FROZEN_T */
  const double *pah_rows;      /* device [n_pah][n_cells][n_lambda] re-emission
                                  CDF rows, required when PAH species exist */
  mcrt_trace_rec *trace;       /* device [n_packets * trace_cap] or NULL */
  int32_t *trace_len;          /* device [n_packets] */
  int32_t trace_cap;
  int32_t pad;
  void *peel_queue;            /* device, peel_capacity * MCRT_PEEL_REC_BYTES, for MCRT_FLAG_PEEL */
  uint64_t peel_capacity;      /* records */
  void *jrec_ws;               /* device workspace of mcrt_jrec_ws_bytes(jrec_capacity) bytes for the
                                  deferred path tally, or NULL for direct atomic adds */
  uint64_t jrec_capacity;      /* path-segment records the workspace holds */
  hipEvent_t kernel_begin;     /* optional (NULL): events recorded on the stream right before and */
  hipEvent_t kernel_end;       /* right after the transport kernel itself, to time it alone */
} mcrt_run_opts;

/* Byte offsets of the tables inside the tables buffer (for inspection). */
typedef struct {
  uint64_t nu, dnu, src_cdf, kext, albedo, gpar, sp_cdf, Tk, E, R, Bt, Wt, xk;
  uint64_t kext32, g32, rho_h32, level, leaf_lo, binfo, pah_slot, scratch, total;
} mcrt_table_layout;

int32_t mcrt_version(void);

/* Size of the tables buffer for a description (no device work). */
int32_t mcrt_tables_bytes(const mcrt_desc *desc, uint64_t *bytes);

/* Validates the description on the host and copies it. */
int32_t mcrt_ctx_create(const mcrt_desc *desc, mcrt_ctx **out);
void mcrt_ctx_destroy(mcrt_ctx *ctx);
const char *mcrt_last_error(const mcrt_ctx *ctx);
int32_t mcrt_table_layout_get(const mcrt_ctx *ctx, mcrt_table_layout *out);

/* Paper Sec. 2: an absorbed packet raises the energy of its cell by eps and
 * with it the cell's temperature, and leaves again at a new frequency drawn
 * from the emission of the cell at the temperature before the absorption
 * (the difference spectrum, without the Bjorkman & Wood correction); the star
 * emits the packets.  These tables carry that arithmetic for the transport.
 * Builds, in FP64 on the device, every table of the method into `tables`
 * (caller-owned, >= mcrt_tables_bytes): bin frequencies and widths, the
 * source CDF over bins, extinction/albedo, the species choice CDF per bin,
 * E_s(T_k) = 4 pi sum_j kabs_s B_j(T_k) dnu_j on the log T grid and the
 * difference-emissivity rows R_{s,k}(j) (CDF over j of
 * kabs_s [B_j(T_{k+1}) - B_j(T_k)] dnu_j), leaf levels and FP32 copies.
 * Blocks once, before any table kernel runs, to check the device inputs:
 * MCRT_E_NUMERIC for NaN/inf/negative opacities or densities, wavelengths not
 * positive and increasing, or |g| >= 1; MCRT_E_INVALID for a grid whose
 * entries are out of range, whose child nodes do not follow their parent, or
 * which is deeper than max_level.  The table kernels then run asynchronously.
 * The source spectrum is fixed here (teff); lum and pos are read per run. */
int32_t mcrt_build_tables(mcrt_ctx *ctx, const mcrt_source *src, void *tables,
                          uint64_t tables_bytes, hipStream_t stream);

/* Sets (copies, validates) the observers of the escape images used by the
 * following runs; n_obs = 0 turns them off.  Host only, no device work. */
int32_t mcrt_set_observers(mcrt_ctx *ctx, const mcrt_observers *obs);

/* Transports packets with ids [first_id, first_id + n_packets) (paper Sec. 2)
 * and adds their tallies.  Random numbers: Philox4x32-10 keyed by seed,
 * counter (id_lo, id_hi, event, 0|1).  Requires mcrt_build_tables; requires
 * tallies->image when observers are set; MCRT_FLAG_PEEL requires observers,
 * tallies->peel, peel_queue and peel_capacity >= 1. */
int32_t mcrt_run(mcrt_ctx *ctx, uint64_t first_id, uint64_t n_packets,
                 const mcrt_run_opts *opts, const mcrt_tallies *tallies,
                 hipStream_t stream);

/* Paper Sec. 2: the energy eps of each packet absorbed in a cell raises the
 * cell's energy, and accordingly its temperature: the temperature is the one
 * at which the cell emits what it absorbed.
 * Equilibrium temperature of every (cell, equilibrium species): solves
 * nabs * eps = rho V E_s(T) for T in [T_lo, T_hi] in FP64 (bracket from the
 * E table, safeguarded Newton on the exact bin sum).  nabs == 0 gives T_lo;
 * PAH species give 0.  T_out: device [n_cells * n_species] double. */
int32_t mcrt_temperatures(mcrt_ctx *ctx, const uint64_t *nabs, uint64_t n_total,
                          double *T_out, hipStream_t stream);

/* Path-length mean intensity (Lucy 1999):
 * J_nu[c][j] = eps * dq * jq[j][c] / (4 pi V_c dnu_j), erg s^-1 cm^-2 Hz^-1 sr^-1.
 * J_out: device [n_cells * n_lambda] float. */
int32_t mcrt_mean_intensity(mcrt_ctx *ctx, const uint64_t *jq, uint64_t n_total,
                            float *J_out, hipStream_t stream);

/* Dust mass of every leaf, rho_c V_c (g), V_c = base_size^3 2^(-3 level_c):
 * the weight of a cell's per-gram emission in sums over the grid (the band
 * powers of the PAH iteration, pah_band_power).  Requires mcrt_build_tables.
 * mass_out: device double [n_cells]. */
int32_t mcrt_cell_mass(mcrt_ctx *ctx, double *mass_out, hipStream_t stream);

/* Optically thin field of the source at every leaf centre, the starting
 * field of the PAH iteration (no dust in the way):
 * J_nu[c][j] = L w_j / (16 pi^2 r_c^2 dnu_j), w_j the source's share of bin j,
 * r_c the distance from the source to the leaf centre, at least half the leaf
 * side.  J_out: device float [n_cells * n_lambda]. */
int32_t mcrt_thin_field(mcrt_ctx *ctx, float *J_out, hipStream_t stream);

/* Deferred path-length tally (TALLY_J with mcrt_run_opts.jrec_ws): instead of
 * one 64-bit atomic add per path segment into the [n_lambda][n_cells] tally,
 * the transport appends a record per segment to the workspace and mcrt_run
 * then adds them with streaming partition passes (two levels for tallies of
 * more than 1536 * 40704 words) and LDS sums, on the same stream; the tally
 * is identical to the one of the atomic path (integer sums).  Segments beyond
 * jrec_capacity records are added directly (still exact).  The workspace also
 * keeps per-bucket record totals from run to run: a run that continues the
 * last one of the context on the same workspace (the next packet ids, same
 * seed, n_total and capacity) sizes its partition from them instead of
 * counting its records (a matter of speed only: the tally stays exact).
 * Runs that overlap on one workspace race.  Workspace bytes for a capacity
 * (16 bytes per record plus small tables): *bytes;
 * MCRT_E_INVALID for capacity outside [4096, 2^35],
 * MCRT_E_UNSUPPORTED when the grid is deeper than 7 levels or the tally has
 * more than 2^20 * 40704 words.  No device work. */
int32_t mcrt_jrec_ws_bytes(const mcrt_ctx *ctx, uint64_t capacity, uint64_t *bytes);

/* Images through a telescope (paper Sec. 4, Fig. 2: the instrument's point
 * spread function, 50 mas at 10 um).  Each of the n_images [npix][npix]
 * images in `image` (device, uint64 sums such as tallies->peel or
 * tallies->image) is multiplied by `scale` and convolved with a Gaussian of
 * full width at half maximum fwhm_pix pixels (sigma = fwhm / (2 sqrt(2 ln 2))),
 * truncated to |dx|, |dy| <= r = mcrt_psf_radius(fwhm_pix) = ceil(3 sigma) and
 * normalised to unit sum over that square (the 2-D weights are the outer
 * product of the 1-D ones); pixels outside an image count as zero, so flux
 * closer than r to the edge is partly lost.  fwhm_pix = 0 copies the scaled
 * image.  weights: device double [2 r + 1] scratch, receives the 1-D weights.
 * out: device double [n_images][npix][npix].  Returns MCRT_E_INVALID for
 * null pointers, npix outside 1..4096 or fwhm_pix outside
 * [0, MCRT_PSF_MAX_FWHM]; asynchronous on stream. */
#define MCRT_PSF_MAX_FWHM 32.0
int32_t mcrt_psf_radius(double fwhm_pix);
int32_t mcrt_image_psf(const uint64_t *image, int32_t n_images, int32_t npix, double scale,
                       double fwhm_pix, double *weights, double *out, hipStream_t stream);

/* mcrt_image_psf without the weights argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * forbid allocation): the 2 r + 1 weights go to a static device array of
 * MCRT_PSF_STATIC_TAPS doubles (1 KiB) that each device holds from the
 * library's load to the end of the process; its address is looked up once per
 * device, on the first call with that device current.  Allocates nothing and
 * calls no allocating routine.  Same arguments, results and errors as
 * mcrt_image_psf, plus MCRT_E_CAPACITY if 2 r + 1 exceeded
 * MCRT_PSF_STATIC_TAPS (no fwhm_pix in range does: r <= 41) and MCRT_E_HIP if
 * the array's address cannot be obtained.  Every call on one device shares
 * that array (it keeps the last call's weights, each call rewrites all it
 * reads): calls that overlap in time on one device, e.g. on two streams,
 * race and must be ordered by the caller. */
#define MCRT_PSF_STATIC_TAPS 128
int32_t mcrt_image_psf_static(const uint64_t *image, int32_t n_images, int32_t npix, double scale,
                              double fwhm_pix, double *out, hipStream_t stream);

/* Copies the MCRT_N_COUNTERS counters of `tallies` to host memory and waits
 * for the stream (so for every launch queued on it before). */
int32_t mcrt_read_counters_sync(const mcrt_tallies *tallies, uint64_t *host_out, hipStream_t stream);

/* Random-access microbenchmark defining the achievable ceiling of the
 * transport kernel's memory traffic.  mode 0: ceil(n_ops / threads) * threads
 * 64-bit atomic adds (+1) to uniformly random slots of table[n_slots]
 * (device, caller-owned, contents incremented); mode 1: as many random 4-byte
 * loads from loads[n_load] (device), sink (device, 1 float) keeps them live.
 * The number of operations actually issued is n_ops rounded up to a multiple
 * of 16 * 256 * (compute units).  Asynchronous on stream. */
int32_t mcrt_bench_random(uint64_t *table, uint64_t n_slots, const float *loads, uint64_t n_load,
                          uint64_t n_ops, uint64_t seed, int32_t mode, float *sink,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
