/*
 * pah.h -- C ABI of the transiently heated PAH emission step (MI355X).
 *
 * Paper: PAHs with 30 and 200 C atoms, 17 Lorentzian emission bands (Sec. 1);
 * their temperature distribution P(T) depends on both strength and hardness of
 * the radiation field (Sec. 4, Fig. 3), so the emission of a cell follows from
 * the steady state of the molecule's enthalpy states, not from one temperature.
 *
 * The exact solver (pah_solve_exact), per cell and in FP64:
 *   states: M enthalpy bins with centres U_i = U(T_i);
 *   heating (photon absorption; cross-section and field constant per
 *     wavelength bin, photons of bin j carrying E_j = h nu_j): the
 *     N_j = 4 pi C_j J_j dnu_j / E_j photons per second of bin j take state i
 *     to x = U_i + E_j, shared between the bin centres U_k <= x < U_{k+1} with
 *     weights (U_{k+1} - x)/(U_{k+1} - U_k) on k and (x - U_k)/(U_{k+1} - U_k)
 *     on k+1 (mean gain exactly E_j; the share left on k = i is no
 *     transition); jumps to or past the top centre land in the top bin;
 *   cooling: continuous, to the next lower bin, A_{i-1,i} =
 *     4 pi sum_j C_j B_j(T_i) dnu_j / (U_i - U_{i-1});
 *   steady state: P_f A_{f-1,f} = sum_{i<f} P_i sum_{k>=f} A_{k,i}, P_0 = 1,
 *     normalised to sum 1;
 *   outputs per cell (erg/s per molecule): n_bands band powers
 *     sum_{i>=1} P_i 4 pi sum_j Cband_b(j) B_j(T_i) dnu_j, then n_lambda
 *     continuum powers 4 pi Ccont(j) B_j(T_i) dnu_j summed the same way
 *     (the ground bin emits nothing: it has no lower state).
 *   With Cband summed over bands plus Ccont equal to C, the outputs add up to
 *   the absorbed power 4 pi sum_j C_j J_j dnu_j whenever no jump passes the
 *   top bin (the deficit is the energy of such jumps above U_{M-1}).
 * Conventions (device arrays caller-owned, async on the stream, error codes)
 * are those of mcrt.h.
 */
#ifndef PAH_H
#define PAH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pah_ctx pah_ctx;

typedef struct {
  int32_t M;                  /* enthalpy bins, >= 3 */
  int32_t n_lambda;           /* wavelength bins, >= 2; 6 M + 13 n_lambda <= 16246 */
  int32_t n_bands;            /* emission bands, 0..64 */
  int32_t pad;
  const double *T;            /* device [M] bin temperatures (K), increasing */
  const double *U;            /* device [M] bin enthalpies (erg), increasing */
  const double *lambda_um;    /* device [n_lambda] bin centres, increasing */
  const double *cabs;         /* device [n_lambda] absorption cross-section, cm^2 */
  const double *cband;        /* device [n_bands * n_lambda] band parts of cabs */
  const double *ccont;        /* device [n_lambda] non-band part of cabs */
} pah_desc;

/* Bytes of the cell-independent tables (no device work). */
int32_t pah_tables_bytes(const pah_desc *desc, uint64_t *bytes);
int32_t pah_ctx_create(const pah_desc *desc, pah_ctx **out);
void pah_ctx_destroy(pah_ctx *ctx);
const char *pah_last_error(const pah_ctx *ctx);

/* Builds the cell-independent tables in FP64 on the device: bin frequencies,
 * widths and photon energies, 1 / (U_f - U_{f-1}), the count m(f,i) of
 * wavelength bins whose photons lift state i to U_f or beyond, cooling rates
 * and the emission of every output at every state temperature.
 * tables: device, >= pah_tables_bytes. */
int32_t pah_build_tables(pah_ctx *ctx, void *tables, uint64_t tables_bytes, hipStream_t stream);

/* Exact steady-state P(T) and emission for n cells.
 * J: device [n][n_lambda] mean intensity J_nu (erg s^-1 cm^-2 Hz^-1 sr^-1),
 *    float when j_is_f32 != 0, else double.
 * out: device [n][n_bands + n_lambda] double (see the header comment).
 * P_out: device [n][M] double or NULL.  pabs_out: device [n] double or NULL,
 *    the absorbed power 4 pi sum_j cabs_j J_j dnu_j.  Needs no scratch memory. */
int32_t pah_solve_exact(pah_ctx *ctx, const void *J, int32_t j_is_f32, int64_t n, double *out,
                        double *P_out, double *pabs_out, hipStream_t stream);

/* Re-emission CDF rows for PAH absorption in the transport (paper Sec. 2: an
 * absorbed packet is re-emitted at a new frequency; for PAHs the frequency
 * follows the molecule's emission spectrum).  Per cell c and bin j: the
 * continuum power out[c][n_bands + j] plus each band power out[c][b] spread
 * over the bins in proportion to cband_b(j) dnu_j; rows[c] is the running sum
 * normalised to end at exactly 1.  out: device double [n][n_bands + n_lambda]
 * (as from pah_solve_exact); rows: device double [n][n_lambda], the layout of
 * one PAH species' slice of mcrt_run_opts.pah_rows. */
int32_t pah_build_rows(pah_ctx *ctx, const double *out, int64_t n, double *rows, hipStream_t stream);

/* Emitted band powers of the model, the quantity whose change between
 * transport passes ends the PAH iteration (paper Sec. 2 with Sec. 1: PAH
 * emission in the Monte Carlo loop; the field of one pass sets the emission
 * the next pass re-emits from):
 * bp_out[b] = sum_c weight[c] out[c][b] for the n_bands bands, FP64, summed
 * in a fixed order (the same result on every call).  With weight the cell's
 * dust mass (mcrt_cell_mass) and out per molecule, bp is the band power up to
 * the constant number of molecules per gram.  out: device double
 * [n][n_bands + n_lambda]; weight: device double [n]; bp_out: device double
 * [n_bands].  Uses a 128 KiB region of the tables buffer for partial sums, so
 * calls on one context must not overlap in time. */
int32_t pah_band_power(pah_ctx *ctx, const double *out, int64_t n, const double *weight, double *bp_out,
                       hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the exact step: a perceptron n_in -> n_h -> n_h -> n_out
 * with SiLU activations, z = W x + b per layer (W stored [out][in]).
 * Inputs (n_in = n_lambda + 1), standardised: the share of the absorbed power
 * in each wavelength bin, f_j = C_j J_j dnu_j / sum C J dnu (the emission per
 * absorbed power is linear in these in the single-photon regime), and
 * log10 P_abs (P_abs = 4 pi sum C J dnu, the field strength); outputs
 * standardised log10(F_q / P_abs) per output q.  Products run on
 * the matrix cores with bfloat16 operands (round to nearest even) and FP32
 * accumulation; weights keep FP32 masters, updated by Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected), and bfloat16 working copies.
 * All state lives in one caller-owned device buffer of pah_mlp_state_bytes;
 * `batch` bounds the rows of one forward/backward call.
 * ------------------------------------------------------------------------ */
typedef struct pah_mlp pah_mlp;

int32_t pah_mlp_state_bytes(int32_t n_in, int32_t n_h, int32_t n_out, int32_t batch, uint64_t *bytes);
int32_t pah_mlp_create(int32_t n_in, int32_t n_h, int32_t n_out, int32_t batch, void *state,
                       uint64_t state_bytes, pah_mlp **out);
void pah_mlp_destroy(pah_mlp *m);
const char *pah_mlp_last_error(const pah_mlp *m);

/* Byte offsets inside the state buffer (for inspection), in this order:
 * params, grads, adam_m, adam_v, n_params (a count), then element offsets of
 * W1 b1 W2 b2 W3 b3 inside a parameter block, then byte offsets of the bf16
 * weights W1 W2 W3, x_mu x_sd x_lo x_hi y_mu y_sd, activations X Z1 H1 Z2 H2
 * Y dY dZ2 dZ1, loss, packed inference weights, total.  off: host array of
 * >= 32 entries. */
int32_t pah_mlp_offsets(const pah_mlp *m, uint64_t *off, int32_t n_off);

/* Copies FP32 parameters (device, flat [W1 b1 W2 b2 W3 b3]) into the masters,
 * zeroes the Adam moments and refreshes the bfloat16 copies. */
int32_t pah_mlp_load(pah_mlp *m, const float *params, hipStream_t stream);

/* Normalisation (device FP32 arrays): input mean, sd, and the standardised
 * training range [x_lo, x_hi] per input; output mean and sd per output. */
int32_t pah_mlp_set_norm(pah_mlp *m, const float *x_mu, const float *x_sd, const float *x_lo,
                         const float *x_hi, const float *y_mu, const float *y_sd, hipStream_t stream);

/* Training pairs from exactly solved cells: x = the input features above,
 * y = log10 max(out / pabs, 1e-20), into X [n][n_in] and Y [n][n_out]
 * (device FP32, caller-owned); then the per-column mean and sd (floored at
 * 1e-3) of both are stored as the network's normalisation, X and Y are
 * standardised in place and the standardised range of X is recorded.
 * J: device float [n][n_lambda]; out, pabs: as returned by pah_solve_exact;
 * ctx: the PAH model (its tables built) the network is for. */
int32_t pah_mlp_prepare(pah_mlp *m, const pah_ctx *ctx, const float *J, const double *out,
                        const double *pabs, int64_t n, float *X, float *Y, hipStream_t stream);

/* Forward pass on standardised inputs X [n][n_in] (device FP32, rounded to
 * bfloat16), writing standardised outputs Y [n][n_out] (device FP32); n <= batch. */
int32_t pah_mlp_forward(pah_mlp *m, const float *X, int32_t n, float *Y, hipStream_t stream);

/* One training step on a batch: forward, mean-squared-error loss against
 * standardised targets T [n][n_out], backward into the grads block, and (if
 * lr != 0) an Adam update with step count `step` (>= 1). */
int32_t pah_mlp_train_step(pah_mlp *m, const float *X, const float *T, int32_t n, float lr,
                           int32_t step, hipStream_t stream);

/* Surrogate emission for n cells from their fields J (device float
 * [n][n_lambda]): out (device double [n][n_bands + n_lambda]) as the exact
 * solver defines it, pabs (device double [n]), and ood (device uint8 [n]):
 * bit 0 set when a standardised input lies more than in_margin outside the
 * training range, bit 1 when the emitted total differs from P_abs by more than
 * balance_tol (relative).  A cell with no absorbed power gets its exact
 * answer, out = 0 (the molecule stays in the ground state, which emits
 * nothing), and no flag.  The network must match the PAH model's shape and
 * the PAH tables must be built. */
int32_t pah_surrogate_infer(pah_mlp *m, const pah_ctx *ctx, const float *J, int64_t n, double *out,
                            uint8_t *ood, double *pabs, float in_margin, float balance_tol,
                            hipStream_t stream);

/* Exact solution for the flagged cells only: every cell c with ood[c] != 0
 * is solved by the exact solver and its row of out overwritten.  The flagged
 * cells are gathered on the device into idx (device int64 [n + 1]; idx[n]
 * receives their count), so no host round trip is needed. */
int32_t pah_exact_fallback(pah_ctx *ctx, const float *J, int64_t n, const uint8_t *ood,
                           double *out, int64_t *idx, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
