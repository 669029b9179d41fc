/*
 * pah.h -- C ABI of the transiently heated PAH emission step (MI355X).
 *
 * Paper: PAHs with 30 and 200 C atoms, 17 Lorentzian emission bands (Sec. 1);
 * their temperature distribution P(T) depends on both strength and hardness of
 * the radiation field (Sec. 4, Fig. 3), so the emission of a cell follows from
 * the steady state of the molecule's enthalpy states, not from one temperature.
 *
 * The exact solver (pah_solve_exact), per cell and in FP64:
 *   states: M enthalpy bins, centres U_i = U(T_i), edges halfway between
 *     centres (bin 0 starts at U_0; the top bin ends half a step above U_{M-1});
 *   heating (photon absorption, cross-section and field constant per
 *     wavelength bin): A_{f,i} = dU_f 4 pi C(E) J_nu(E) / (h E), E = U_f - U_i,
 *     zero outside the wavelength grid; the top bin takes every jump at or above
 *     its lower edge (integral of the same rate density);
 *   cooling: continuous, to the next lower bin, A_{i-1,i} =
 *     4 pi sum_j C_j B_j(T_i) dnu_j / (U_i - U_{i-1});
 *   steady state: P_f A_{f-1,f} = sum_{i<f} P_i sum_{k>=f} A_{k,i}, P_0 = 1,
 *     normalised to sum 1;
 *   outputs per cell (erg/s per molecule): n_bands band powers
 *     sum_{i>=1} P_i 4 pi sum_j Cband_b(j) B_j(T_i) dnu_j, then n_lambda
 *     continuum powers 4 pi Ccont(j) B_j(T_i) dnu_j summed the same way
 *     (the ground bin emits nothing: it has no lower state).
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
  int32_t M;                  /* enthalpy bins, 3..4096 */
  int32_t n_lambda;           /* wavelength bins, 2..4096 */
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

/* Builds the cell-independent tables in FP64 on the device: bin frequencies
 * and widths, heating weights dU_f 4 pi / (h E) with the wavelength bin of
 * each jump E, the top-bin integrals, cooling rates and the emission of every
 * output at every state temperature.  tables: device, >= pah_tables_bytes. */
int32_t pah_build_tables(pah_ctx *ctx, void *tables, uint64_t tables_bytes, hipStream_t stream);

/* Workspace (device, caller-owned) needed by pah_solve_exact. */
int32_t pah_workspace_bytes(const pah_ctx *ctx, uint64_t *bytes);

/* Exact steady-state P(T) and emission for n cells.
 * J: device [n][n_lambda] mean intensity J_nu (erg s^-1 cm^-2 Hz^-1 sr^-1),
 *    float when j_is_f32 != 0, else double.
 * out: device [n][n_bands + n_lambda] double (see the header comment).
 * P_out: device [n][M] double or NULL.  pabs_out: device [n] double or NULL,
 *    the absorbed power 4 pi sum_j cabs_j J_j dnu_j.
 * ws: device workspace of >= pah_workspace_bytes. */
int32_t pah_solve_exact(pah_ctx *ctx, const void *J, int32_t j_is_f32, int64_t n, double *out,
                        double *P_out, double *pabs_out, void *ws, uint64_t ws_bytes,
                        hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
