/*
 * lecqmc.h -- C ABI of the MI355X (gfx950) hot path of linear-scaling
 * canonical-ensemble determinant QMC (arXiv 2601.08552).
 *
 * The library samples (eta, s) with probability proportional to
 *   |W(eta, s)|,  W = prod_sigma det[P_sigma^T B^sigma(beta, 0) P_sigma]
 * (main text Eq. (1)) for the Hubbard-type Hamiltonian
 *   H = sum_b h_b (c_i^dag c_j + h.c.) + sum_i eps_i n_i + U sum_i n_iu n_id
 * (main text, Hubbard model; SM Sec. III for the flat-band chain) at fixed
 * particle numbers N_up, N_dn, and accumulates equal-time estimators.
 *
 * Conventions fixed by this ABI:
 *   B_l = E_K D_l,   D_l^sigma = diag(exp(sigma lambda s_{l,i} - dtau eps_i)),
 *   cosh(lambda) = exp(dtau U / 2) (Ising decoupling in the spin channel),
 *   E_K = e^{-dtau K_0} e^{-dtau K_1} ... e^{-dtau K_{C-1}} over the bond
 *   colours supplied by the caller (bonds of one colour never share a site).
 *   L_tau = beta / dtau slices; a QR stabilisation every n_stab slices
 *   (SM Sec. I.A: n = L_tau / tau_w stabilisation steps; the last block may
 *   be shorter).  W excludes the configuration-independent factor
 *   2^{-N L_tau} e^{-beta U (N_up + N_dn) / 2}.
 *
 * One sweep = (i) left-stack build, (ii) forward pass over all L_tau slices
 * with one Ising flip attempt per (slice, site) accepted on the Ne x Ne
 * determinant ratio with a rank-1 update (main text, auxiliary-field
 * updates), QR stabilisation at block ends, (iii) Ne_sigma particle-hole
 * swap attempts per spin at tau = beta, each a removal (permutation +
 * Givens retriangulation, SM Sec. I.B) followed by an addition (one-column
 * propagation + Gram-Schmidt per level, SM Sec. I.A).
 *
 * Errors: every int-returning call returns 0 on success or a negative code
 * below; lecqmc_last_error() gives a message (thread-local).  Calls on one
 * walker are not thread-safe; distinct walkers may be used from different
 * threads only through distinct contexts.  Kernels are launched on the
 * context's stream; lecqmc_sweep / lecqmc_sweep_batch return without
 * waiting, every call that returns data to the host synchronises the stream.
 */
#ifndef LECQMC_H
#define LECQMC_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define LECQMC_OK 0
#define LECQMC_EINVAL (-1)    /* bad sizes or arguments (message says which)          */
#define LECQMC_ENOMEM (-2)    /* device footprint over the context budget (refused)   */
#define LECQMC_EUNSTABLE (-3) /* singular inverse or QR breakdown (kept), or a wrap error above
                                 wrap_tol on a measuring sweep (reported once by the next
                                 call that reads the walker's status; the walker stays valid) */
#define LECQMC_EDEVICE (-4)   /* HIP runtime error                                    */
#define LECQMC_ESTATE (-5)    /* call not valid in the walker's state                 */

#define LECQMC_FP64 0         /* all arithmetic in FP64                               */
#define LECQMC_MIXED 1        /* mixed precision: the slice propagation (Slater blocks,
                                 stored left states, Fock columns: E_K and D_l) is
                                 stored and computed in FP32 between stabilisations;
                                 QR and Gram matrices, Ne x Ne inverses and
                                 determinants, log-weights, flip and swap ratios
                                 and the right stack stay FP64                    */
#define LECQMC_NO_FOCK 1      /* flags: skip the particle-hole swap phase             */
#define LECQMC_NO_FLIPS 2     /* flags: skip the Ising flips (fields frozen)          */

#define LECQMC_MAX_NE 256     /* largest particle number per spin handled on device  */
#define LECQMC_STATIC_MAX_WALKERS 1024 /* walkers per lecqmc_sweep_batch_static call  */

/* Flags not provided: a symmetric checkerboard split (e^{-dtau K/2} on both
 * sides of D_l) and heat-bath acceptance.  The paper fixes neither; the
 * build implements one reading of each (asymmetric product, Metropolis on
 * |r|), the one its oracle pins. */

typedef struct lecqmc_ctx lecqmc_ctx;
typedef struct lecqmc_walker lecqmc_walker;

/* Lattice (host arrays, copied at walker creation; caller keeps ownership). */
typedef struct {
  int32_t n_sites, n_bonds, n_colors;
  const int32_t *bond_i, *bond_j, *bond_color; /* [n_bonds]; colours 0..n_colors-1 */
  const double *bond_h;                        /* [n_bonds] hopping element h_ij   */
  const double *onsite;                        /* [n_sites] eps_i, or NULL          */
  const int32_t *sublattice;                   /* [n_sites] 0..n_sublattices-1, or NULL */
  int32_t n_sublattices, n_cells;              /* n_cells <= 0 means n_sites        */
} lecqmc_lattice;

typedef struct {
  double U, beta, dtau;
  int32_t n_stab;           /* slices per QR stabilisation, >= 1              */
  int32_t n_up, n_dn;       /* 0..min(n_sites, LECQMC_MAX_NE)                 */
  uint64_t seed, walker_id; /* key of the counter-based generator             */
  int32_t precision;        /* LECQMC_FP64 or LECQMC_MIXED                    */
  int32_t flags;            /* LECQMC_NO_FOCK | LECQMC_NO_FLIPS               */
  double wrap_tol;          /* largest |A_wrap - A_fresh| on the diagonal at a
                               measured stabilisation boundary (SM Sec. I.A: the
                               wrapped and the freshly recomputed Green's
                               functions agree); <= 0: 1e-8 (FP64) or 1e-4
                               (LECQMC_MIXED)                                   */
} lecqmc_params;

typedef struct {
  int64_t flip_attempts, flip_accepts;   /* cumulative since creation          */
  int64_t swap_attempts, swap_accepts;
  double max_wrap_err;                   /* max over block starts               */
  double logw_drift;                     /* max |tracked - fresh| log W at beta */
  int64_t qr_shifted;                    /* QR calls that needed the shifted retry */
  uint64_t sweeps;                       /* sweep counter                       */
  int64_t near_ties;                     /* flip and swap decisions u < |r| with
                                            |u - |r|| < 1e-9: a rounding change of r
                                            that size could have reversed them   */
} lecqmc_sweep_stats;

/* Context: device ordinal, a borrowed hipStream_t (NULL = the library makes
 * its own, non-blocking, default priority), and the device-memory budget used
 * for admission (0 = no limit).  Work of different contexts (streams) may
 * overlap on the device. */
int lecqmc_ctx_create(int device, void *hip_stream_or_null, size_t hbm_budget_bytes, lecqmc_ctx **out);
/* Destroying a context that still owns walkers fails with LECQMC_ESTATE. */
int lecqmc_ctx_destroy(lecqmc_ctx *ctx);
int lecqmc_ctx_synchronize(lecqmc_ctx *ctx);
/* Non-blocking: 1 when all work queued on the context's stream has finished,
 * 0 while some is still running, a negative code on a device error. */
int lecqmc_ctx_query(lecqmc_ctx *ctx);
size_t lecqmc_ctx_bytes_in_use(const lecqmc_ctx *ctx);
/* Per-phase device timing: when enabled, every sweep records HIP events on
 * the context's stream around its three launches (left stack, forward pass,
 * Fock phase).  phase_times synchronises, returns the summed milliseconds and
 * launch counts per phase since the last call, and resets them. */
int lecqmc_ctx_set_timing(lecqmc_ctx *ctx, int32_t enable);
int lecqmc_ctx_phase_times(lecqmc_ctx *ctx, double ms[3], int64_t counts[3]);

/* Device bytes one walker needs (right and left stacks dominate:
 * 2 * (2 n + 1) * N * Ne * 8 bytes plus the stored left states,
 * 2 * L_tau * N * Ne * 8 bytes, or * 4 bytes with LECQMC_MIXED); 0 if the
 * input is invalid. */
size_t lecqmc_footprint_bytes(const lecqmc_lattice *lat, const lecqmc_params *par);

/* Create a walker (one Markov chain over (eta, s), main text Eq. (1)):
 * copies the lattice, builds the model tables (checkerboard bond
 * exponentials; Ising decoupling cosh(lambda) = exp(dtau U / 2)), draws the
 * fields (fields_or_null == NULL: s = +1 iff U(INIT_FIELD) < 1/2) and the
 * occupation (NULL: partial Fisher-Yates shuffle) or takes the given ones,
 * fields [L_tau][n_sites] int8 (+-1), occupations int32 distinct sites in
 * column order.  Computes the fresh weight.  -2 if over the budget. */
int lecqmc_create_walker(lecqmc_ctx *ctx, const lecqmc_lattice *lat, const lecqmc_params *par,
                         const int8_t *fields_or_null, const int32_t *occ_up_or_null,
                         const int32_t *occ_dn_or_null, lecqmc_walker **out);
int lecqmc_destroy_walker(lecqmc_walker *w);

/* n_sweeps full sweeps (left stack, forward pass with the Ising-field
 * updates by the fast update of the projector-like sweep, main text
 * "Ensemble constrained quantum Monte Carlo"; QR every n_stab slices, SM
 * Sec. I.A; N_sigma particle-hole swaps per spin, main text "Linear ensemble
 * constrained quantum Monte Carlo", SM Secs. I.A and I.B).  do_measure != 0
 * accumulates estimators at the interior stabilisation boundaries (tau =
 * beta when there is one block) and runs the wrap check against wrap_tol.
 * Returns without waiting: device errors and LECQMC_EUNSTABLE surface on the
 * next call that reads the walker back. */
int lecqmc_sweep(lecqmc_walker *w, int32_t n_sweeps, int32_t do_measure);
/* The same for n walkers of one context in one launch per phase; shapes
 * may differ between walkers.  FP64 and mixed-precision walkers may be
 * combined: each precision gets its own launch per phase.  ws holds n
 * distinct walkers (LECQMC_EINVAL if one appears twice).  The descriptor
 * array is grown with hipMalloc when n exceeds every earlier call's. */
int lecqmc_sweep_batch(lecqmc_walker *const *ws, int32_t n, int32_t n_sweeps, int32_t do_measure);
/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): lecqmc_sweep_batch with the walker descriptors
 * staged in a fixed per-device array of LECQMC_STATIC_MAX_WALKERS entries
 * (528 KiB, held until the process ends) instead of a grown allocation.  It
 * calls no hipMalloc, hipFree or other allocating routine and records no
 * phase timing.  n > LECQMC_STATIC_MAX_WALKERS: LECQMC_EINVAL.  All calls on
 * one GPU share that array: calls that overlap on one GPU (from contexts on
 * different streams) race, so callers serialise them. */
int lecqmc_sweep_batch_static(lecqmc_walker *const *ws, int32_t n, int32_t n_sweeps, int32_t do_measure);

/* A fixed batch of walkers of one context (uneven shapes and precisions
 * allowed): their descriptors are uploaded once, so lecqmc_batch_sweep only
 * launches kernels on the context's stream -- no allocation, copy,
 * synchronisation or event -- and a call may be recorded into a HIP graph
 * by stream capture and replayed (every replay advances the walkers by the
 * recorded sweeps; the sweep counters live on the device).  Phase timing
 * (lecqmc_ctx_set_timing) does not see these sweeps.  A walker of a live
 * batch cannot be destroyed (LECQMC_ESTATE); destroy the batch first. */
typedef struct lecqmc_batch lecqmc_batch;
int lecqmc_batch_create(lecqmc_walker *const *ws, int32_t n, lecqmc_batch **out);
int lecqmc_batch_sweep(lecqmc_batch *b, int32_t n_sweeps, int32_t do_measure);
int lecqmc_batch_destroy(lecqmc_batch *b);

/* Flip-chain shape of a walker.  tile = register tile T in {1, 2, 4}: the
 * Ne x Ne inverse of each spin is held in registers of one wavefront, which
 * needs Ne <= 8T; tile = 0: the inverse stays in LDS (any Ne); tile = 9:
 * delayed (submatrix) updates of chunks of sites on the vector units (any
 * Ne, chunk <= 16); tile = 10: delayed updates of 16-site chunks on the FP64
 * matrix cores (Ne <= 128, chunk 16; the decisions by Gauss-Jordan sweeps of
 * the chunk's 16 x 16 matrix, the inverse by the Woodbury identity).
 * chunk = sites staged per step of the chain: 4, 8, 16 or 32.  New walkers take a default
 * by Ne, or the shape an earlier lecqmc_autotune chose in the same context
 * for the same (n_sites, n_up, n_dn, precision).  Every shape samples the
 * same chain: the tile changes only the rounding order of the ratio sums,
 * the chunk changes nothing.  A walker's shape is its own: walkers of
 * different shapes in one batch keep theirs.  set_shape returns
 * LECQMC_EINVAL for a shape that is not valid for the walker's Ne and
 * LECQMC_ESTATE while the walker belongs to a batch. */
int lecqmc_get_shape(const lecqmc_walker *w, int32_t *tile, int32_t *chunk);
int lecqmc_set_shape(lecqmc_walker *w, int32_t tile, int32_t chunk);
/* Autotuner: runs one whole forward pass of the given walkers for every
 * (tile, chunk) that is valid for them (walkers of one precision launched
 * together), times each walker by the device wall clock inside the kernel,
 * and restores every walker's fields and scalars after each candidate.  The
 * walkers of one (n_sites, n_up, n_dn, precision) key then all get the shape
 * with the least total time over them, and the context records it for that
 * key.  The Markov chains are not advanced.  Outputs, arrays of n that may
 * each be NULL: the chosen tile and chunk, and the walker's forward-pass
 * milliseconds with them.  Synchronises the context's stream and allocates
 * device memory for the saved state.  LECQMC_ESTATE if a walker belongs to
 * a batch. */
int lecqmc_autotune(lecqmc_walker *const *ws, int32_t n, int32_t *tile_out, int32_t *chunk_out,
                    double *fwd_ms_out);

/* Fresh log|W| and sign from the current (eta, s), main text Eq. (1): the
 * right chain B_s(beta, 0) P with a QR every n_stab slices (SM Sec. I.A,
 * B_i Q_{i-1} = Q_i V_i), log|W| = sum log V_jj + log|det(P^T Q_n)| summed
 * over both spins; FP64 whatever the walker's precision. */
int lecqmc_log_weight(lecqmc_walker *w, double *log_abs_w, int32_t *sign);
/* Weight carried by the chain (updated by every accepted move, reset to the
 * fresh value at tau = beta of each sweep). */
int lecqmc_tracked_weight(lecqmc_walker *w, double *log_abs_w, int32_t *sign);

/* Sign-weighted accumulators since the last reset (Wick contractions of
 * A = Phi_R (Phi_L Phi_R)^{-1} Phi_L at the measurement boundaries; the q = 0
 * structure factors as defined with main text Fig. 4); layout:
 *  [0] sum sign  [1] number of measurements  [2] double occupancy per site
 *  [3] kinetic energy per site  [4] S_par(q=0) = (1/L_c) sum_ij <SxSx+SySy>
 *  [5] S_zz(q=0) total  [6] onsite energy per site  [7] density per site
 *  [8 .. 8+ns^2) S_zz(q=0)_ab  [.. +ns^2) S_par(q=0)_ab
 *  if n_sites <= 64: <S_i.S_j> (N^2), <n_i n_j> (N^2), <n_i up> (N), <n_i dn> (N)
 * every entry already multiplied by the sign of the configuration. */
int64_t lecqmc_obs_size(const lecqmc_walker *w);
int lecqmc_measure(lecqmc_walker *w, double *out, int64_t n);
/* Status-reading calls (lecqmc_measure, lecqmc_get_stats, lecqmc_log_weight,
 * lecqmc_tracked_weight and the parity surface) fill their outputs and then
 * return LECQMC_EUNSTABLE when a sweep since the last report found a wrap
 * error above wrap_tol (or a singular inverse). */
int lecqmc_reset_measure(lecqmc_walker *w);
int lecqmc_get_stats(lecqmc_walker *w, lecqmc_sweep_stats *st);

/* State access (host buffers): fields [L_tau][N], occupations, sweep counter. */
int lecqmc_get_state(lecqmc_walker *w, int8_t *fields, int32_t *occ_up, int32_t *occ_dn,
                     uint64_t *sweep_counter);
int lecqmc_set_state(lecqmc_walker *w, const int8_t *fields, const int32_t *occ_up,
                     const int32_t *occ_dn, uint64_t sweep_counter);

/* Parity surface (fresh recomputation, small systems):
 * G_ij = <c_i c_j^dag> at slice boundary b in 0..L_tau, N x N row-major,
 * G = I - Phi_R (Phi_L Phi_R)^{-1} Phi_L with Phi_R = B_s(b, 0) P and
 * Phi_L = P^T B_s(beta, b), both stabilised by QR (SM Sec. I.A).  The N x N
 * device staging is allocated for the call only and counts against the
 * context's budget while it lives (LECQMC_ENOMEM if it does not fit). */
int lecqmc_green(lecqmc_walker *w, int32_t boundary, int32_t spin, double *G);
/* r = r_up r_dn for flipping s_{slice, site} (slice 0-based), not applied:
 * r_sigma = 1 + Delta_sigma [Phi_R M^{-1} Phi_L]_{site, site} at the flip
 * point of the slice (the fast-update ratio, main text "Ensemble constrained
 * quantum Monte Carlo"). */
int lecqmc_flip_ratio(lecqmc_walker *w, int32_t slice, int32_t site, double *ratio);
/* Remove occupied index k_index of spin, add empty site j: weight ratio of the
 * composite move (removal by column permutation and Givens retriangulation,
 * SM Sec. I.B; addition by one-column propagation and Gram-Schmidt at every
 * level, SM Sec. I.A and main text eq. ratio) from a fresh right stack, not
 * applied. */
int lecqmc_swap_ratio(lecqmc_walker *w, int32_t spin, int32_t k_index, int32_t j_site, double *ratio);

const char *lecqmc_last_error(void);

/* ---- Constrained-path (phaseless) inner walk (SM Sec. VI) ----------------
 * Two-stage sampling of the canonical partition function: Fock states eta are
 * drawn with the trial weight W_T(eta) = <eta| e^{-beta H_0} |eta> (the chain
 * of a walker with U = 0), and for one eta a population of random walkers
 * estimates
 *   R(eta) = E_s[ prod_sigma det(P^T B^sigma(s) P) ] / W_T(eta)
 * (s uniform over the Ising fields) as the product of the overlap ratios of
 * each walker with the backward trial state <eta| e^{-(beta - tau_l) H_0}, the
 * fields drawn site by site with rank-1 (Sherman-Morrison) updates and the
 * phaseless cut max(0, r).  H_0 is the lattice's one-body part (hopping and
 * onsite energies); the interaction is the Ising decoupling of U with the
 * walker parameters' U, beta, dtau and n_stab (QR of each walker every n_stab
 * slices).
 * Field draws of walker slot a at slice l, site i: the counter-based uniform
 * of (seed, walker_id = a, stream 7, sweep = tag, l - 1, i); the comb after
 * slice l: (seed, 0, stream 8, tag, l - 1, 0).
 *   mode LECQMC_CP_IMPORTANCE: s = +1 with probability
 *     max(0, r(+1)) / (max(0, r(+1)) + max(0, r(-1))), the weight times
 *     (max(0, r(+1)) + max(0, r(-1))) / 2;
 *   mode LECQMC_CP_FREE: s = +1 with probability 1/2, the weight times
 *     max(0, r(s)).
 * A walker whose factor is 0 is dead (weight 0) and draws nothing more.
 * pc_every > 0: after every pc_every-th slice (not the last) a comb with one
 * uniform draw replaces the population by n_walkers copies chosen in
 * proportion to their weights, each of weight 1; the log of the mean weight
 * is accumulated into the estimate.
 * Limits: FP64 only; n_up, n_dn <= 64 (the inverses live in LDS). */
#define LECQMC_CP_IMPORTANCE 0
#define LECQMC_CP_FREE 1
typedef struct lecqmc_cp lecqmc_cp;
/* The Fock state (occ_up[n_up], occ_dn[n_dn], distinct sites) and the
 * population size; builds the U = 0 trial walker and its backward trial
 * states (device memory counted against the context budget).  EINVAL on bad
 * arguments or limits, ENOMEM over the budget. */
int lecqmc_cp_create(lecqmc_ctx *ctx, const lecqmc_lattice *lat, const lecqmc_params *par,
                     const int32_t *occ_up, const int32_t *occ_dn, int32_t n_walkers, int32_t mode,
                     int32_t pc_every, lecqmc_cp **out);
/* One inner walk from Phi = P_eta over all slices; *log_r = log of the
 * estimate of R(eta) (-inf when every walker died).  Blocks until done. */
int lecqmc_cp_run(lecqmc_cp *cp, uint32_t tag, double *log_r);
/* After a run: walker slot a's log weight (since the last comb), the sum of
 * the log probabilities of its draws (importance mode; copied with it by a
 * comb) and its field path (host int8[L_tau][n_sites], 0 where it drew
 * nothing); any pointer may be NULL. */
int lecqmc_cp_walker(lecqmc_cp *cp, int32_t a, double *log_w, double *log_q, int8_t *fields);
/* After a run: accumulated log mean weight of the combs, walkers cut by the
 * constraint, walkers alive at the end. */
int lecqmc_cp_stats(lecqmc_cp *cp, double *log_pc, int64_t *cuts, int32_t *alive);
int lecqmc_cp_destroy(lecqmc_cp *cp);

#ifdef __cplusplus
}
#endif
#endif
