/*
 * lecqmc_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the
 * canonical-ensemble (fixed particle number) determinant QMC of
 * "Linear Canonical-Ensemble Quantum Monte Carlo" (arXiv 2601.08552).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header or table
 * with the HIP implementation.
 *
 * What it computes (main text Eq. (1) and SM Sec. I):
 *   weight  W(eta, s) = prod_sigma det[P_sigma^T B^sigma(beta,0) P_sigma],
 *   B^sigma(beta,0) = B_L ... B_1,   B_l = E_K D_l^sigma,
 *   D_l^sigma = diag(exp(sigma*lambda*s_{l,i} - dtau*eps_i)), cosh(lambda) = exp(dtau*U/2)
 *   (discrete Ising decoupling of U n_up n_dn, spin channel),
 *   E_K = e^{-dtau K_0} ... e^{-dtau K_{C-1}} (checkerboard colours given as input).
 * Markov chain: HS-field flips with a rank-1 (Sherman-Morrison) update of the
 * Ne x Ne inverse (main text, "Ensemble constrained QMC"), QR stabilisation
 * every n_stab slices, and particle-hole swap moves built from the paper's
 * stabilized QR update (SM Sec. I.A adding, Sec. I.B removing).
 */
#ifndef LECQMC_ORACLE_H
#define LECQMC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_sites, n_bonds, n_colors;
  const int32_t *bond_i, *bond_j, *bond_color;
  const double *bond_h;      /* hopping matrix element h_ij (-t for the usual -t) */
  const double *onsite;      /* eps_i, may be NULL */
  const int32_t *sublattice; /* may be NULL = one sublattice */
  int32_t n_sublattices, n_cells;
} orc_lattice;

typedef struct {
  double U, beta, dtau;
  int32_t n_stab, n_up, n_dn;
  uint64_t seed, walker_id;
  int32_t flags;             /* ORC_NO_FOCK | ORC_NO_FLIPS */
  double wrap_tol;
} orc_params;

enum { ORC_NO_FOCK = 1, ORC_NO_FLIPS = 2 };

/* RNG streams of the counter-based generator */
enum { ORC_S_FLIP = 1, ORC_S_SWAP_K = 2, ORC_S_SWAP_J = 3, ORC_S_SWAP_ACC = 4,
       ORC_S_INIT_FIELD = 5, ORC_S_INIT_OCC = 6, ORC_S_CP_FIELD = 7, ORC_S_CP_COMB = 8 };

typedef struct orc_walker orc_walker;

typedef struct {
  int64_t flip_attempts, flip_accepts;
  int64_t swap_attempts, swap_accepts;
  double max_wrap_err;       /* max_i |A_wrap_ii - A_fresh_ii| at block starts */
  double logw_drift;         /* |tracked log W - fresh log W| at tau = beta */
  int64_t near_ties;         /* flip and swap decisions with |u - |r|| < 1e-9 */
} orc_stats;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform double in [0,1) for (stream, sweep, a, b) of walker (seed, walker_id). */
double orc_uniform(uint64_t seed, uint64_t walker_id, uint32_t stream, uint32_t sweep,
                   uint32_t a, uint32_t b);

/* Returns NULL on invalid input (message in orc_last_error()). */
orc_walker *orc_create(const orc_lattice *lat, const orc_params *par,
                       const int8_t *fields_or_null, const int32_t *occ_up_or_null,
                       const int32_t *occ_dn_or_null);
void orc_destroy(orc_walker *w);
const char *orc_last_error(void);

int orc_sweep(orc_walker *w, int32_t n_sweeps, int32_t do_measure);
int orc_log_weight(orc_walker *w, double *log_abs_w, int32_t *sign);
int orc_tracked_weight(const orc_walker *w, double *log_abs_w, int32_t *sign);
int orc_get_state(const orc_walker *w, int8_t *fields, int32_t *occ_up, int32_t *occ_dn,
                  uint64_t *sweep_counter);
int orc_set_state(orc_walker *w, const int8_t *fields, const int32_t *occ_up,
                  const int32_t *occ_dn, uint64_t sweep_counter);
/* G_ij = <c_i c_j^dag> at the slice boundary b (0..L_tau), N x N row-major. */
int orc_green(orc_walker *w, int32_t boundary, int32_t spin, double *G);
/* r = r_up * r_dn for flipping s_{slice,site} in the current configuration. */
int orc_flip_ratio(orc_walker *w, int32_t slice, int32_t site, double *ratio);
/* Remove occupied index k of spin, add site j (must be empty); ratio only.
 * Builds a fresh right stack from the current state first. */
int orc_swap_ratio(orc_walker *w, int32_t spin, int32_t k_index, int32_t j_site, double *ratio);
/* Same move, committed unconditionally (for the stack/inverse invariants).
 * Returns the ratio; the right stack and the inverse stay readable. */
int orc_swap_commit(orc_walker *w, int32_t spin, int32_t k_index, int32_t j_site, double *ratio);
/* Right stack access (after a sweep or a swap): Q_k (N x Ne_sigma), V_k (Ne x Ne),
 * and the inverse of P^T Q_n. */
int orc_right_stack(const orc_walker *w, int32_t spin, int32_t level, double *Q, double *V);
int orc_inverse(const orc_walker *w, int32_t spin, double *Minv);
int orc_n_blocks(const orc_walker *w);

int64_t orc_obs_size(const orc_walker *w);
int orc_measure(const orc_walker *w, double *out);
int orc_reset_measure(orc_walker *w);
int orc_get_stats(const orc_walker *w, orc_stats *st);

/* ---- Constrained-path (phaseless) inner walk, SM Sec. VI ----------------
 * For one Fock state eta (occ_up, occ_dn), a population of n_walkers random
 * walkers propagates Phi = P_eta through B_l(s) = E_K D0 F_l(s) with the
 * Ising fields drawn site by site; each walker's weight is the product of
 * the overlap ratios with the backward trial state <eta| e^{-(beta-tau) H_0}
 * under the phaseless cut max(0, r).  log_r = log of the estimate of
 *   R(eta) = E_{s uniform}[ prod_sigma det(P^T B^sigma(s) P) ] / W_T(eta).
 * Field draws: orc_uniform(seed, walker slot, ORC_S_CP_FIELD, tag, l - 1, i);
 * comb draw after slice l: orc_uniform(seed, 0, ORC_S_CP_COMB, tag, l - 1, 0). */
enum { ORC_CP_IMPORTANCE = 0, ORC_CP_FREE = 1 };
typedef struct orc_cp orc_cp;
orc_cp *orc_cp_create(const orc_lattice *lat, const orc_params *par, const int32_t *occ_up,
                      const int32_t *occ_dn, int32_t n_walkers, int32_t mode, int32_t pc_every);
void orc_cp_destroy(orc_cp *c);
int orc_cp_run(orc_cp *c, uint32_t tag, double *log_r);
/* final log weight, sum of log p(s) of its draws (importance mode), and its
 * field path [L][N] of walker slot a after the last run */
int orc_cp_walker(const orc_cp *c, int32_t a, double *log_w, double *log_q, int8_t *fields);
int orc_cp_stats(const orc_cp *c, double *log_pc, int64_t *cuts, int32_t *alive);

#ifdef __cplusplus
}
#endif
#endif
