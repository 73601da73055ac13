/*
 * lecqmc_oracle.c -- plain, slow, single-threaded FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see lecqmc_oracle.h).  Every routine follows the
 * paper's steps in the paper's order, written for a reader who checks it
 * against the text: no blocking, no fusion, no reordering, no BLAS.
 *
 * Storage: every Slater block is an N x Ne row-major array.  The left state
 * Phi_L (Ne x N) is kept transposed, X = Phi_L^T (N x Ne).
 * Slices are numbered l = 1..L (B_l = E_K D_l), blocks k = 1..n with block k
 * holding slices (k-1)*n_stab+1 .. min(k*n_stab, L).
 */
#include "lecqmc_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 as published by Salmon et al. */
/* (SC'11): 10 rounds of two 32x32->64 multiplies with the round constants    */
/* M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the Weyl key increments               */
/* W0 = 0x9E3779B9, W1 = 0xBB67AE85.                                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* counter = (a, b, sweep, stream | walker_id << 8), key = seed (lo, hi);
 * the double takes the top 53 bits of (out0 << 32 | out1). */
double orc_uniform(uint64_t seed, uint64_t walker_id, uint32_t stream, uint32_t sweep,
                   uint32_t a, uint32_t b) {
  uint32_t ctr[4] = {a, b, sweep, (stream & 0xffu) | (uint32_t)((walker_id & 0xffffffu) << 8)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  uint64_t bits = ((uint64_t)o[0] << 32) | o[1];
  return (double)(bits >> 11) * (1.0 / 9007199254740992.0);
}

/* floor(u * n) clamped to n - 1 */
static int pick(double u, int n) {
  int v = (int)floor(u * (double)n);
  return v >= n ? n - 1 : v;
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra (textbook)                                          */
/* ------------------------------------------------------------------------ */

/* Thin Householder QR of X (n x m row-major, n >= m): X = Q R with Q (n x m)
 * orthonormal columns and R (m x m) upper triangular with diag(R) >= 0. */
static void qr_pos(const double *X, int n, int m, double *Q, double *R) {
  double *A = malloc(sizeof(double) * (size_t)n * (m ? m : 1));
  double *vs = malloc(sizeof(double) * (size_t)n * (m ? m : 1));
  double *taus = malloc(sizeof(double) * (m ? m : 1));
  memcpy(A, X, sizeof(double) * (size_t)n * m);
  for (int j = 0; j < m; ++j) {
    double nrm = 0.0;
    for (int i = j; i < n; ++i) nrm += A[(size_t)i * m + j] * A[(size_t)i * m + j];
    nrm = sqrt(nrm);
    double *v = vs + (size_t)j * n;
    if (nrm == 0.0) { taus[j] = 0.0; continue; }
    double ajj = A[(size_t)j * m + j];
    double alpha = (ajj >= 0.0) ? -nrm : nrm;
    double vn2 = 0.0;
    for (int i = j; i < n; ++i) {
      v[i] = A[(size_t)i * m + j] - (i == j ? alpha : 0.0);
      vn2 += v[i] * v[i];
    }
    taus[j] = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    for (int c = j; c < m; ++c) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += v[i] * A[(size_t)i * m + c];
      for (int i = j; i < n; ++i) A[(size_t)i * m + c] -= taus[j] * d * v[i];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < m; ++c) R[i * m + c] = (c >= i) ? A[(size_t)i * m + c] : 0.0;
  /* Q = H_0 H_1 ... H_{m-1} [I_m; 0] */
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < m; ++c) Q[(size_t)i * m + c] = (i == c) ? 1.0 : 0.0;
  for (int j = m - 1; j >= 0; --j) {
    if (taus[j] == 0.0) continue;
    double *v = vs + (size_t)j * n;
    for (int c = 0; c < m; ++c) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += v[i] * Q[(size_t)i * m + c];
      for (int i = j; i < n; ++i) Q[(size_t)i * m + c] -= taus[j] * d * v[i];
    }
  }
  for (int j = 0; j < m; ++j) {
    if (R[j * m + j] < 0.0) {
      for (int c = 0; c < m; ++c) R[j * m + c] = -R[j * m + c];
      for (int i = 0; i < n; ++i) Q[(size_t)i * m + j] = -Q[(size_t)i * m + j];
    }
  }
  free(A); free(vs); free(taus);
}

/* Inverse, log|det| and sign of det of an m x m matrix by LU with partial
 * pivoting.  Returns 0, or -1 if a pivot is exactly zero. */
static int lu_inverse(const double *M, int m, double *Minv, double *logabs, int *sign) {
  *logabs = 0.0; *sign = 1;
  if (m == 0) return 0;
  double *A = malloc(sizeof(double) * m * m);
  int *piv = malloc(sizeof(int) * m);
  memcpy(A, M, sizeof(double) * m * m);
  for (int i = 0; i < m; ++i) piv[i] = i;
  int s = 1;
  for (int c = 0; c < m; ++c) {
    int p = c;
    double best = fabs(A[c * m + c]);
    for (int r = c + 1; r < m; ++r)
      if (fabs(A[r * m + c]) > best) { best = fabs(A[r * m + c]); p = r; }
    if (best == 0.0) { free(A); free(piv); *logabs = -INFINITY; *sign = 0; return -1; }
    if (p != c) {
      for (int x = 0; x < m; ++x) { double t = A[c * m + x]; A[c * m + x] = A[p * m + x]; A[p * m + x] = t; }
      int t = piv[c]; piv[c] = piv[p]; piv[p] = t;
      s = -s;
    }
    for (int r = c + 1; r < m; ++r) {
      double f = A[r * m + c] / A[c * m + c];
      A[r * m + c] = f;
      for (int x = c + 1; x < m; ++x) A[r * m + x] -= f * A[c * m + x];
    }
  }
  double la = 0.0;
  for (int c = 0; c < m; ++c) {
    la += log(fabs(A[c * m + c]));
    if (A[c * m + c] < 0.0) s = -s;
  }
  /* solve A x = e_col for each column (with the row permutation) */
  double *y = malloc(sizeof(double) * m);
  for (int col = 0; col < m; ++col) {
    for (int r = 0; r < m; ++r) y[r] = (piv[r] == col) ? 1.0 : 0.0;
    for (int r = 0; r < m; ++r)
      for (int x = 0; x < r; ++x) y[r] -= A[r * m + x] * y[x];
    for (int r = m - 1; r >= 0; --r) {
      for (int x = r + 1; x < m; ++x) y[r] -= A[r * m + x] * y[x];
      y[r] /= A[r * m + r];
    }
    for (int r = 0; r < m; ++r) Minv[r * m + col] = y[r];
  }
  free(y); free(A); free(piv);
  *logabs = la; *sign = s;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Walker                                                                    */
/* ------------------------------------------------------------------------ */
struct orc_walker {
  int N, L, nstab, nblk, ncol, nsub, ncells, nbonds;
  int ne[2];
  double dtau, U, lambda;
  uint64_t seed, wid;
  uint32_t sweep;
  int flags;
  /* model tables: bonds grouped by colour */
  int *col_start;            /* [ncol + 1] */
  int *cb_i, *cb_j;          /* [nbonds] */
  double *cb_diag, *cb_off;  /* cosh(dtau h), -sinh(dtau h) */
  double *bond_h;            /* h per grouped bond */
  double *eps_fac;           /* exp(-dtau eps_i), [N] */
  double *eps;               /* eps_i or zeros */
  int *sub;                  /* [N] */
  int8_t *s;                 /* [L][N] */
  int *occ[2];
  /* right stack and inverse at tau = beta */
  double *RQ[2], *RV[2], *Minv[2];
  int stack_valid;
  double logw; int sign;
  /* measurement accumulators */
  double *obs; int64_t nobs;
  orc_stats st;
};

static int block_first(const orc_walker *w, int k) { return (k - 1) * w->nstab + 1; }
static int block_last(const orc_walker *w, int k) {
  int e = k * w->nstab;
  return e > w->L ? w->L : e;
}

/* spin index sp = 0 (up, sigma = +1) or 1 (down, sigma = -1) */
static double dfac(const orc_walker *w, int l, int i, int sp) {
  double sigma = sp == 0 ? 1.0 : -1.0;
  return exp(sigma * w->lambda * (double)w->s[(size_t)(l - 1) * w->N + i]) * w->eps_fac[i];
}

/* apply one colour's bond exponentials to the rows of X (N x m):
 * [x_i; x_j] <- [d o; o d] [x_i; x_j], o -> -o for the inverse. */
static void colour_apply(const orc_walker *w, double *X, int m, int c, int inverse) {
  for (int b = w->col_start[c]; b < w->col_start[c + 1]; ++b) {
    int i = w->cb_i[b], j = w->cb_j[b];
    double d = w->cb_diag[b], o = inverse ? -w->cb_off[b] : w->cb_off[b];
    for (int a = 0; a < m; ++a) {
      double xi = X[(size_t)i * m + a], xj = X[(size_t)j * m + a];
      X[(size_t)i * m + a] = d * xi + o * xj;
      X[(size_t)j * m + a] = o * xi + d * xj;
    }
  }
}
/* X <- E_K X, E_K = e^{-dtau K_0} ... e^{-dtau K_{C-1}}: colour C-1 acts first */
static void ek_left(const orc_walker *w, double *X, int m) {
  for (int c = w->ncol - 1; c >= 0; --c) colour_apply(w, X, m, c, 0);
}
/* X <- E_K^T X: colour 0 acts first */
static void ekT_left(const orc_walker *w, double *X, int m) {
  for (int c = 0; c < w->ncol; ++c) colour_apply(w, X, m, c, 0);
}
/* X <- E_K^{-T} X = e^{dtau K_0} ... e^{dtau K_{C-1}} X: colour C-1 acts first */
static void ekinvT_left(const orc_walker *w, double *X, int m) {
  for (int c = w->ncol - 1; c >= 0; --c) colour_apply(w, X, m, c, 1);
}
static void diag_left(const orc_walker *w, double *X, int m, int l, int sp, int inverse) {
  for (int i = 0; i < w->N; ++i) {
    double f = dfac(w, l, i, sp);
    if (inverse) f = 1.0 / f;
    for (int a = 0; a < m; ++a) X[(size_t)i * m + a] *= f;
  }
}

static void fill_P(const orc_walker *w, int sp, double *X) {
  int m = w->ne[sp];
  memset(X, 0, sizeof(double) * (size_t)w->N * m);
  for (int a = 0; a < m; ++a) X[(size_t)w->occ[sp][a] * m + a] = 1.0;
}

/* M = X^T Y (X: N x m, Y: N x m) */
static void xty(const double *X, const double *Y, int N, int m, double *M) {
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      double acc = 0.0;
      for (int i = 0; i < N; ++i) acc += X[(size_t)i * m + a] * Y[(size_t)i * m + b];
      M[a * m + b] = acc;
    }
}

/* Right chain from P: B_l ... B_1 P with QR at every block end, storing the
 * stack (Q_k, V_k), k = 1..nblk.  Used by log_weight and swap_ratio.       */
static void right_stack(orc_walker *w, int sp) {
  int N = w->N, m = w->ne[sp];
  double *Phi = malloc(sizeof(double) * (size_t)N * (m ? m : 1));
  fill_P(w, sp, Phi);
  for (int k = 1; k <= w->nblk; ++k) {
    for (int l = block_first(w, k); l <= block_last(w, k); ++l) {
      diag_left(w, Phi, m, l, sp, 0);
      ek_left(w, Phi, m);
    }
    double *Q = w->RQ[sp] + (size_t)(k - 1) * N * m, *V = w->RV[sp] + (size_t)(k - 1) * m * m;
    qr_pos(Phi, N, m, Q, V);
    memcpy(Phi, Q, sizeof(double) * (size_t)N * m);
  }
  free(Phi);
}

/* M = P^T Q_n, its inverse; returns log|det M|, sign */
static void inverse_at_beta(orc_walker *w, int sp, double *logabs, int *sign) {
  int N = w->N, m = w->ne[sp];
  (void)N;
  double *M = malloc(sizeof(double) * (m ? m * m : 1));
  const double *Qn = w->RQ[sp] + (size_t)(w->nblk - 1) * w->N * m;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) M[a * m + b] = Qn[(size_t)w->occ[sp][a] * m + b];
  lu_inverse(M, m, w->Minv[sp], logabs, sign);
  free(M);
}

/* log W = sum_sigma [ sum_k sum_j log V_k,jj + log|det P^T Q_n| ] (SM Sec. I.A:
 * the weight factorises into det[P^T Q] det[R], R = V_n ... V_1). */
static void fresh_weight(orc_walker *w, double *logabs, int *sign) {
  double la = 0.0; int sg = 1;
  for (int sp = 0; sp < 2; ++sp) {
    int m = w->ne[sp];
    right_stack(w, sp);
    for (int k = 0; k < w->nblk; ++k)
      for (int j = 0; j < m; ++j) la += log(w->RV[sp][(size_t)k * m * m + j * m + j]);
    double l2; int s2;
    inverse_at_beta(w, sp, &l2, &s2);
    la += l2; sg *= s2;
  }
  w->stack_valid = 1;
  *logabs = la; *sign = sg;
}

static int obs_layout_size(int N, int nsub) {
  return 8 + 2 * nsub * nsub + (N <= 64 ? 2 * N * N + 2 * N : 0);
}

orc_walker *orc_create(const orc_lattice *lat, const orc_params *par,
                       const int8_t *fields, const int32_t *occ_up, const int32_t *occ_dn) {
  if (!lat || !par) { set_err("null argument"); return NULL; }
  int N = lat->n_sites;
  if (N <= 0 || lat->n_bonds < 0 || lat->n_colors < 0) { set_err("bad lattice sizes"); return NULL; }
  if (par->n_up < 0 || par->n_up > N || par->n_dn < 0 || par->n_dn > N) { set_err("particle number out of range"); return NULL; }
  if (par->n_stab <= 0 || par->dtau <= 0.0 || par->beta <= 0.0) { set_err("bad time parameters"); return NULL; }
  double Lf = par->beta / par->dtau;
  int L = (int)llround(Lf);
  if (L <= 0 || fabs(Lf - L) > 1e-9 * (Lf > 1 ? Lf : 1)) { set_err("beta/dtau not integral"); return NULL; }
  for (int b = 0; b < lat->n_bonds; ++b) {
    if (lat->bond_i[b] < 0 || lat->bond_i[b] >= N || lat->bond_j[b] < 0 || lat->bond_j[b] >= N ||
        lat->bond_i[b] == lat->bond_j[b] || lat->bond_color[b] < 0 || lat->bond_color[b] >= lat->n_colors) {
      set_err("bad bond"); return NULL;
    }
  }
  /* colours must be site-disjoint */
  int *seen = calloc(N, sizeof(int));
  for (int c = 0; c < lat->n_colors; ++c) {
    for (int b = 0; b < lat->n_bonds; ++b) {
      if (lat->bond_color[b] != c) continue;
      if (seen[lat->bond_i[b]] == c + 1 || seen[lat->bond_j[b]] == c + 1) { free(seen); set_err("colour with a shared site"); return NULL; }
      seen[lat->bond_i[b]] = c + 1; seen[lat->bond_j[b]] = c + 1;
    }
  }
  free(seen);

  orc_walker *w = calloc(1, sizeof *w);
  w->N = N; w->L = L; w->nstab = par->n_stab; w->nblk = (L + par->n_stab - 1) / par->n_stab;
  w->ncol = lat->n_colors; w->nbonds = lat->n_bonds;
  w->ne[0] = par->n_up; w->ne[1] = par->n_dn;
  w->dtau = par->dtau; w->U = par->U;
  /* Ising decoupling of U n_up n_dn (spin channel): cosh(lambda) = exp(dtau U / 2) */
  w->lambda = acosh(exp(par->dtau * par->U / 2.0));
  w->seed = par->seed; w->wid = par->walker_id; w->flags = par->flags;
  w->nsub = (lat->sublattice && lat->n_sublattices > 0) ? lat->n_sublattices : 1;
  w->ncells = lat->n_cells > 0 ? lat->n_cells : N;

  w->col_start = calloc(w->ncol + 1, sizeof(int));
  w->cb_i = malloc(sizeof(int) * (w->nbonds ? w->nbonds : 1));
  w->cb_j = malloc(sizeof(int) * (w->nbonds ? w->nbonds : 1));
  w->cb_diag = malloc(sizeof(double) * (w->nbonds ? w->nbonds : 1));
  w->cb_off = malloc(sizeof(double) * (w->nbonds ? w->nbonds : 1));
  w->bond_h = malloc(sizeof(double) * (w->nbonds ? w->nbonds : 1));
  int pos = 0;
  for (int c = 0; c < w->ncol; ++c) {
    w->col_start[c] = pos;
    for (int b = 0; b < lat->n_bonds; ++b) {
      if (lat->bond_color[b] != c) continue;
      double h = lat->bond_h[b];
      w->cb_i[pos] = lat->bond_i[b]; w->cb_j[pos] = lat->bond_j[b];
      /* e^{-dtau h (|i><j| + |j><i|)} restricted to {i, j} */
      w->cb_diag[pos] = cosh(par->dtau * h);
      w->cb_off[pos] = -sinh(par->dtau * h);
      w->bond_h[pos] = h;
      ++pos;
    }
  }
  w->col_start[w->ncol] = pos;
  w->eps_fac = malloc(sizeof(double) * N);
  w->eps = calloc(N, sizeof(double));
  w->sub = calloc(N, sizeof(int));
  for (int i = 0; i < N; ++i) {
    w->eps[i] = lat->onsite ? lat->onsite[i] : 0.0;
    w->eps_fac[i] = exp(-par->dtau * w->eps[i]);
    w->sub[i] = lat->sublattice ? lat->sublattice[i] : 0;
    if (w->sub[i] < 0 || w->sub[i] >= w->nsub) { orc_destroy(w); set_err("bad sublattice index"); return NULL; }
  }
  w->s = malloc((size_t)L * N);
  for (int l = 0; l < L; ++l)
    for (int i = 0; i < N; ++i) {
      int8_t v;
      if (fields) v = fields[(size_t)l * N + i] > 0 ? 1 : -1;
      else v = orc_uniform(w->seed, w->wid, ORC_S_INIT_FIELD, 0, (uint32_t)l, (uint32_t)i) < 0.5 ? 1 : -1;
      w->s[(size_t)l * N + i] = v;
    }
  for (int sp = 0; sp < 2; ++sp) {
    int m = w->ne[sp];
    w->occ[sp] = malloc(sizeof(int) * (N + 1));
    const int32_t *given = sp == 0 ? occ_up : occ_dn;
    if (given) {
      char *used = calloc(N, 1);
      for (int a = 0; a < m; ++a) {
        if (given[a] < 0 || given[a] >= N || used[given[a]]) { free(used); orc_destroy(w); set_err("bad occupation list"); return NULL; }
        used[given[a]] = 1; w->occ[sp][a] = given[a];
      }
      free(used);
    } else {
      /* partial Fisher-Yates shuffle of 0..N-1 */
      int *perm = malloc(sizeof(int) * N);
      for (int i = 0; i < N; ++i) perm[i] = i;
      for (int a = 0; a < m; ++a) {
        int j = a + pick(orc_uniform(w->seed, w->wid, ORC_S_INIT_OCC, 0, (uint32_t)sp, (uint32_t)a), N - a);
        int t = perm[a]; perm[a] = perm[j]; perm[j] = t;
        w->occ[sp][a] = perm[a];
      }
      free(perm);
    }
    size_t mm = m ? (size_t)m : 1;
    w->RQ[sp] = malloc(sizeof(double) * (size_t)w->nblk * N * mm);
    w->RV[sp] = malloc(sizeof(double) * (size_t)w->nblk * mm * mm);
    w->Minv[sp] = malloc(sizeof(double) * mm * mm);
  }
  w->nobs = obs_layout_size(N, w->nsub);
  w->obs = calloc(w->nobs, sizeof(double));
  fresh_weight(w, &w->logw, &w->sign);
  return w;
}

void orc_destroy(orc_walker *w) {
  if (!w) return;
  free(w->col_start); free(w->cb_i); free(w->cb_j); free(w->cb_diag); free(w->cb_off);
  free(w->bond_h); free(w->eps_fac); free(w->eps); free(w->sub); free(w->s);
  for (int sp = 0; sp < 2; ++sp) { free(w->occ[sp]); free(w->RQ[sp]); free(w->RV[sp]); free(w->Minv[sp]); }
  free(w->obs);
  free(w);
}

int orc_n_blocks(const orc_walker *w) { return w->nblk; }

/* ------------------------------------------------------------------------ */
/* Left stack (backward build): Y <- P; for k = n..1, for l = last..first of */
/* block k: Y <- D_l E_K^T Y; QR; LS[k-1] = Q.  LS[n] = P.                    */
/* LS[k] spans Phi_L^T at the boundary after slice k*n_stab.                 */
/* ------------------------------------------------------------------------ */
static double *left_stack(const orc_walker *w, int sp) {
  int N = w->N, m = w->ne[sp];
  size_t blk = (size_t)N * (m ? m : 1);
  double *LS = malloc(sizeof(double) * blk * (w->nblk + 1));
  double *Y = malloc(sizeof(double) * blk);
  double *R = malloc(sizeof(double) * (m ? m * m : 1));
  fill_P(w, sp, Y);
  memcpy(LS + (size_t)w->nblk * blk, Y, sizeof(double) * (size_t)N * m);
  for (int k = w->nblk; k >= 1; --k) {
    for (int l = block_last(w, k); l >= block_first(w, k); --l) {
      ekT_left(w, Y, m);
      diag_left(w, Y, m, l, sp, 0);
    }
    double *Q = LS + (size_t)(k - 1) * blk;
    qr_pos(Y, N, m, Q, R);
    memcpy(Y, Q, sizeof(double) * (size_t)N * m);
  }
  free(Y); free(R);
  return LS;
}

/* A = Phi_R Minv Phi_L, i.e. A_ij = <c_j^dag c_i> (N x N) */
static void build_A(int N, int m, const double *PhiR, const double *Minv, const double *X, double *A) {
  double *T = calloc((size_t)N * (m ? m : 1), sizeof(double));
  for (int i = 0; i < N; ++i)
    for (int b = 0; b < m; ++b) {
      double acc = 0.0;
      for (int a = 0; a < m; ++a) acc += PhiR[(size_t)i * m + a] * Minv[a * m + b];
      T[(size_t)i * m + b] = acc;
    }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double acc = 0.0;
      for (int b = 0; b < m; ++b) acc += T[(size_t)i * m + b] * X[(size_t)j * m + b];
      A[(size_t)i * N + j] = acc;
    }
  free(T);
}

/* Equal-time estimators by Wick's theorem from A_sigma (sign-weighted). */
static void measure_point(orc_walker *w, double *const A[2], int sgn) {
  int N = w->N, ns = w->nsub;
  double *o = w->obs;
  double sg = (double)sgn;
  double *Au = A[0], *Ad = A[1];
#define AU(i, j) Au[(size_t)(i) * N + (j)]
#define AD(i, j) Ad[(size_t)(i) * N + (j)]
  o[0] += sg;
  o[1] += 1.0;
  double docc = 0.0, ekin = 0.0, eon = 0.0, dens = 0.0;
  for (int i = 0; i < N; ++i) {
    docc += AU(i, i) * AD(i, i);
    eon += w->eps[i] * (AU(i, i) + AD(i, i));
    dens += AU(i, i) + AD(i, i);
  }
  for (int b = 0; b < w->nbonds; ++b) {
    int i = w->cb_i[b], j = w->cb_j[b];
    ekin += w->bond_h[b] * (AU(i, j) + AU(j, i) + AD(i, j) + AD(j, i));
  }
  o[2] += sg * docc / N;
  o[3] += sg * ekin / N;
  o[6] += sg * eon / N;
  o[7] += sg * dens / N;
  double *szz = o + 8, *spar = o + 8 + ns * ns;
  int full = N <= 64;
  double *ss = o + 8 + 2 * ns * ns, *nn = ss + (size_t)N * N, *nu = nn + (size_t)N * N, *nd = nu + N;
  double szz_tot = 0.0, spar_tot = 0.0;
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      double d = (i == j) ? 1.0 : 0.0;
      double uu = AU(i, i) * AU(j, j) + AU(j, i) * (d - AU(i, j));
      double dd = AD(i, i) * AD(j, j) + AD(j, i) * (d - AD(i, j));
      double ud = AU(i, i) * AD(j, j);
      double du = AD(i, i) * AU(j, j);
      double zz = 0.25 * (uu + dd - ud - du);
      double pm = AU(j, i) * (d - AD(i, j));   /* <S+_i S-_j> */
      double mp = AD(j, i) * (d - AU(i, j));   /* <S-_i S+_j> */
      double xy = 0.5 * (pm + mp);
      szz[w->sub[i] * ns + w->sub[j]] += sg * zz / w->ncells;
      spar[w->sub[i] * ns + w->sub[j]] += sg * xy / w->ncells;
      szz_tot += zz; spar_tot += xy;
      if (full) {
        ss[(size_t)i * N + j] += sg * (zz + xy);
        nn[(size_t)i * N + j] += sg * (uu + dd + ud + du);
      }
    }
    if (full) { nu[i] += sg * AU(i, i); nd[i] += sg * AD(i, i); }
  }
  o[4] += sg * spar_tot / w->ncells;
  o[5] += sg * szz_tot / w->ncells;
#undef AU
#undef AD
}

/* ------------------------------------------------------------------------ */
/* Particle-hole swap: removal (SM Sec. I.B) then addition (SM Sec. I.A)     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int ne, m, k, j;           /* m = ne - 1 particles after the removal */
  int *perm;                 /* column order after U: [0..k-1, k+1..ne-1, k] */
  double *gc, *gs;           /* [nblk][ne] rotation (c, s) for rows (r, r+1), r = k..ne-2 */
  double *Vp;                /* [nblk][ne*ne] V_i' = G_i H_i */
  double *Mp;                /* ne*ne  (P U)^T Q_n' inverse = G_n M^{-1} U */
  double *Mred;              /* m*m reduced inverse */
  double *q;                 /* [nblk][N] new orthonormal columns q_i */
  double *v;                 /* [nblk][m] projection coefficients */
  double *rho;               /* [nblk] */
  double *acol, *brow;       /* block-inverse vectors, m each */
  double schur;
  double log_abs_r; int sign_r; int zero;
} swap_work;

static void sw_free(swap_work *x) {
  free(x->perm); free(x->gc); free(x->gs); free(x->Vp); free(x->Mp); free(x->Mred);
  free(x->q); free(x->v); free(x->rho); free(x->acol); free(x->brow);
}

/* apply G_i (rows r = k..ne-2 in order) to a vector y of length ne */
static void givens_vec(const swap_work *x, int lvl, double *y) {
  const double *c = x->gc + (size_t)lvl * x->ne, *s = x->gs + (size_t)lvl * x->ne;
  for (int r = x->k; r <= x->ne - 2; ++r) {
    double a = y[r], b = y[r + 1];
    y[r] = c[r] * a + s[r] * b;
    y[r + 1] = -s[r] * a + c[r] * b;
  }
}
/* apply G_i^T to a vector: transposed rotations, r = ne-2 down to k */
static void givensT_vec(const swap_work *x, int lvl, double *y) {
  const double *c = x->gc + (size_t)lvl * x->ne, *s = x->gs + (size_t)lvl * x->ne;
  for (int r = x->ne - 2; r >= x->k; --r) {
    double a = y[r], b = y[r + 1];
    y[r] = c[r] * a - s[r] * b;
    y[r + 1] = s[r] * a + c[r] * b;
  }
}

/* Compute the swap ratio from the current right stack and inverse. */
static void swap_compute(orc_walker *w, int sp, int k, int j, swap_work *x) {
  int N = w->N, ne = w->ne[sp], m = ne - 1, n = w->nblk;
  memset(x, 0, sizeof *x);
  x->ne = ne; x->m = m; x->k = k; x->j = j;
  x->perm = malloc(sizeof(int) * ne);
  for (int c = 0, p = 0; c < ne; ++c) if (c != k) x->perm[p++] = c;
  x->perm[ne - 1] = k;
  x->gc = calloc((size_t)n * ne, sizeof(double));
  x->gs = calloc((size_t)n * ne, sizeof(double));
  x->Vp = malloc(sizeof(double) * (size_t)n * ne * ne);
  x->Mp = malloc(sizeof(double) * ne * ne);
  x->Mred = malloc(sizeof(double) * (m ? m * m : 1));
  x->q = malloc(sizeof(double) * (size_t)n * N);
  x->v = calloc((size_t)n * (m ? m : 1), sizeof(double));
  x->rho = malloc(sizeof(double) * n);
  x->acol = calloc(m ? m : 1, sizeof(double));
  x->brow = calloc(m ? m : 1, sizeof(double));

  /* --- removal: permutation U, then Givens retriangulation at every level --- */
  double log_rne = 0.0; int sign_rne = 1;
  for (int lvl = 0; lvl < n; ++lvl) {
    const double *V = w->RV[sp] + (size_t)lvl * ne * ne;
    double *H = x->Vp + (size_t)lvl * ne * ne;
    if (lvl == 0) {
      /* H = V_1 U (move column k last) */
      for (int r = 0; r < ne; ++r)
        for (int c = 0; c < ne; ++c) H[r * ne + c] = V[r * ne + x->perm[c]];
    } else {
      /* H = V_i G_{i-1}^T: column rotations r = k..ne-2 in order */
      memcpy(H, V, sizeof(double) * ne * ne);
      const double *c = x->gc + (size_t)(lvl - 1) * ne, *s = x->gs + (size_t)(lvl - 1) * ne;
      for (int r = k; r <= ne - 2; ++r)
        for (int row = 0; row < ne; ++row) {
          double a = H[row * ne + r], b = H[row * ne + r + 1];
          H[row * ne + r] = c[r] * a + s[r] * b;
          H[row * ne + r + 1] = -s[r] * a + c[r] * b;
        }
    }
    /* retriangulate the upper-Hessenberg part with row rotations */
    double *c = x->gc + (size_t)lvl * ne, *s = x->gs + (size_t)lvl * ne;
    for (int r = k; r <= ne - 2; ++r) {
      double a = H[r * ne + r], b = H[(r + 1) * ne + r];
      double h = hypot(a, b);
      double cc = 1.0, ss = 0.0;
      if (h != 0.0) { cc = a / h; ss = b / h; }
      c[r] = cc; s[r] = ss;
      for (int col = r; col < ne; ++col) {
        double u = H[r * ne + col], d = H[(r + 1) * ne + col];
        H[r * ne + col] = cc * u + ss * d;
        H[(r + 1) * ne + col] = -ss * u + cc * d;
      }
      H[(r + 1) * ne + r] = 0.0;
    }
    double last = H[(ne - 1) * ne + (ne - 1)];
    log_rne += log(fabs(last));
    if (last < 0.0) sign_rne = -sign_rne;
    if (last == 0.0) x->zero = 1;
  }
  /* M_perm^{-1} = G_n M^{-1} U */
  {
    double *T = malloc(sizeof(double) * ne * ne);
    memcpy(T, w->Minv[sp], sizeof(double) * ne * ne);
    const double *c = x->gc + (size_t)(n - 1) * ne, *s = x->gs + (size_t)(n - 1) * ne;
    for (int r = k; r <= ne - 2; ++r)
      for (int col = 0; col < ne; ++col) {
        double a = T[r * ne + col], b = T[(r + 1) * ne + col];
        T[r * ne + col] = c[r] * a + s[r] * b;
        T[(r + 1) * ne + col] = -s[r] * a + c[r] * b;
      }
    for (int r = 0; r < ne; ++r)
      for (int col = 0; col < ne; ++col) x->Mp[r * ne + col] = T[r * ne + x->perm[col]];
    free(T);
  }
  double mlast = x->Mp[(ne - 1) * ne + (ne - 1)];
  if (mlast == 0.0) x->zero = 1;
  /* removal ratio r_rem = [M_perm^{-1}]_{Ne,Ne} / r_Ne */
  double log_rem = log(fabs(mlast)) - log_rne;
  int sign_rem = (mlast < 0.0 ? -1 : 1) * sign_rne;
  /* reduced inverse (SM Sec. I.B, sub-block extraction) */
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      x->Mred[a * m + b] = x->Mp[a * ne + b] - x->Mp[a * ne + (ne - 1)] * x->Mp[(ne - 1) * ne + b] / mlast;

  /* --- addition of site j to the reduced system, layer by layer --- */
  double *wv = malloc(sizeof(double) * N);
  double *y = malloc(sizeof(double) * ne), *z = malloc(sizeof(double) * ne);
  double log_rho = 0.0;
  for (int i = 0; i < N; ++i) wv[i] = 0.0;
  wv[j] = 1.0;
  for (int lvl = 0; lvl < n && !x->zero; ++lvl) {
    for (int l = block_first(w, lvl + 1); l <= block_last(w, lvl + 1); ++l) {
      diag_left(w, wv, 1, l, sp, 0);
      ek_left(w, wv, 1);
    }
    const double *Q = w->RQ[sp] + (size_t)lvl * N * ne;
    double *vt = x->v + (size_t)lvl * (m ? m : 1);
    for (int pass = 0; pass < 2 && m > 0; ++pass) {
      /* v_pass = (Q_i G_i^T)[:, :m]^T w  =  (G_i Q_i^T w)[:m] */
      for (int a = 0; a < ne; ++a) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += Q[(size_t)i * ne + a] * wv[i];
        y[a] = acc;
      }
      givens_vec(x, lvl, y);
      for (int a = 0; a < ne; ++a) z[a] = (a < m) ? y[a] : 0.0;
      for (int a = 0; a < m; ++a) vt[a] += z[a];
      /* w -= Q_i G_i^T [v; 0] */
      givensT_vec(x, lvl, z);
      for (int i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int a = 0; a < ne; ++a) acc += Q[(size_t)i * ne + a] * z[a];
        wv[i] -= acc;
      }
    }
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) nrm += wv[i] * wv[i];
    nrm = sqrt(nrm);
    x->rho[lvl] = nrm;
    if (!(nrm > 1e-300)) { x->zero = 1; break; }
    double *q = x->q + (size_t)lvl * N;
    for (int i = 0; i < N; ++i) { q[i] = wv[i] / nrm; wv[i] = q[i]; }
    log_rho += log(nrm);
  }
  free(wv); free(y); free(z);
  if (x->zero) { x->log_abs_r = -INFINITY; x->sign_r = 0; return; }
  /* Schur complement s = q_n[j] - (Q^red_n[j,:]) Mred (q_n[occ']) */
  {
    const double *Qn = w->RQ[sp] + (size_t)(n - 1) * N * ne;
    const double *qn = x->q + (size_t)(n - 1) * N;
    double *t = malloc(sizeof(double) * ne);
    for (int a = 0; a < ne; ++a) t[a] = Qn[(size_t)j * ne + a];
    givens_vec(x, n - 1, t);                   /* row j of Q_n G_n^T */
    /* a = Mred P'^T q, b = p^T Q^red Mred */
    for (int a = 0; a < m; ++a) {
      double acc = 0.0;
      for (int b = 0; b < m; ++b) acc += x->Mred[a * m + b] * qn[w->occ[sp][x->perm[b]]];
      x->acol[a] = acc;
    }
    for (int b = 0; b < m; ++b) {
      double acc = 0.0;
      for (int a = 0; a < m; ++a) acc += t[a] * x->Mred[a * m + b];
      x->brow[b] = acc;
    }
    double sch = qn[j];
    for (int a = 0; a < m; ++a) sch -= t[a] * x->acol[a];
    x->schur = sch;
    free(t);
  }
  if (x->schur == 0.0) { x->zero = 1; x->log_abs_r = -INFINITY; x->sign_r = 0; return; }
  /* r = r_rem * r_add, r_add = s * prod_i rho_i (eq. ratio_htp) */
  x->log_abs_r = log_rem + log(fabs(x->schur)) + log_rho;
  x->sign_r = sign_rem * (x->schur < 0.0 ? -1 : 1);
}

/* Commit an accepted swap: new stack, new inverse (block inverse), new occupation. */
static void swap_commit(orc_walker *w, int sp, const swap_work *x) {
  int N = w->N, ne = x->ne, m = x->m, n = w->nblk;
  for (int lvl = 0; lvl < n; ++lvl) {
    double *Q = w->RQ[sp] + (size_t)lvl * N * ne;
    const double *c = x->gc + (size_t)lvl * ne, *s = x->gs + (size_t)lvl * ne;
    for (int i = 0; i < N; ++i) {
      double *row = Q + (size_t)i * ne;
      for (int r = x->k; r <= ne - 2; ++r) {
        double a = row[r], b = row[r + 1];
        row[r] = c[r] * a + s[r] * b;
        row[r + 1] = -s[r] * a + c[r] * b;
      }
      row[ne - 1] = x->q[(size_t)lvl * N + i];
    }
    double *V = w->RV[sp] + (size_t)lvl * ne * ne;
    const double *Vp = x->Vp + (size_t)lvl * ne * ne;
    for (int a = 0; a < ne; ++a)
      for (int b = 0; b < ne; ++b) {
        double val;
        if (a < m && b < m) val = Vp[a * ne + b];
        else if (b == ne - 1 && a < m) val = x->v[(size_t)lvl * (m ? m : 1) + a];
        else if (a == ne - 1 && b == ne - 1) val = x->rho[lvl];
        else val = 0.0;
        V[a * ne + b] = val;
      }
  }
  /* block inverse of the augmented system (SM Sec. I.A) */
  double *Mi = w->Minv[sp];
  double is = 1.0 / x->schur;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) Mi[a * ne + b] = x->Mred[a * m + b] + is * x->acol[a] * x->brow[b];
  for (int a = 0; a < m; ++a) { Mi[a * ne + (ne - 1)] = -is * x->acol[a]; Mi[(ne - 1) * ne + a] = -is * x->brow[a]; }
  Mi[(ne - 1) * ne + (ne - 1)] = is;
  int *occ = w->occ[sp];
  int *nocc = malloc(sizeof(int) * ne);
  for (int a = 0; a < m; ++a) nocc[a] = occ[x->perm[a]];
  nocc[ne - 1] = x->j;
  memcpy(occ, nocc, sizeof(int) * ne);
  free(nocc);
}

static int nth_empty_site(const orc_walker *w, int sp, int nth) {
  char *occd = calloc(w->N, 1);
  for (int a = 0; a < w->ne[sp]; ++a) occd[w->occ[sp][a]] = 1;
  int cnt = 0, site = -1;
  for (int i = 0; i < w->N; ++i)
    if (!occd[i]) { if (cnt == nth) { site = i; break; } ++cnt; }
  free(occd);
  return site;
}

/* ------------------------------------------------------------------------ */
/* One sweep                                                                 */
/* ------------------------------------------------------------------------ */
static void one_sweep(orc_walker *w, int do_measure) {
  int N = w->N, n = w->nblk;
  w->sweep += 1;
  uint32_t sw = w->sweep;
  double *LS[2], *PhiR[2], *X[2], *M[2];
  for (int sp = 0; sp < 2; ++sp) {
    int m = w->ne[sp];
    size_t blk = (size_t)N * (m ? m : 1);
    LS[sp] = left_stack(w, sp);
    PhiR[sp] = malloc(sizeof(double) * blk);
    X[sp] = malloc(sizeof(double) * blk);
    M[sp] = malloc(sizeof(double) * (m ? m * m : 1));
    fill_P(w, sp, PhiR[sp]);
  }
  double *A[2] = {NULL, NULL};
  if (do_measure) { A[0] = malloc(sizeof(double) * (size_t)N * N); A[1] = malloc(sizeof(double) * (size_t)N * N); }
  double *Aw = malloc(sizeof(double) * N);
  double *u = malloc(sizeof(double) * (N + 1)), *wr = malloc(sizeof(double) * (N + 1));
  for (int k = 1; k <= n; ++k) {
    /* fresh left state and inverse at the start of block k */
    int fresh_sign = 1;
    for (int sp = 0; sp < 2; ++sp) {
      int m = w->ne[sp];
      memcpy(X[sp], LS[sp] + (size_t)(k - 1) * N * m, sizeof(double) * (size_t)N * m);
      xty(X[sp], PhiR[sp], N, m, M[sp]);
      double la; int sg;
      lu_inverse(M[sp], m, w->Minv[sp], &la, &sg);
      fresh_sign *= sg;
    }
    if (k > 1 && do_measure) {
      for (int sp = 0; sp < 2; ++sp) build_A(N, w->ne[sp], PhiR[sp], w->Minv[sp], X[sp], A[sp]);
      measure_point(w, A, fresh_sign);
    }
    for (int l = block_first(w, k); l <= block_last(w, k); ++l) {
      for (int sp = 0; sp < 2; ++sp) {
        diag_left(w, PhiR[sp], w->ne[sp], l, sp, 0);
        diag_left(w, X[sp], w->ne[sp], l, sp, 1);
      }
      if (!(w->flags & ORC_NO_FLIPS)) {
        for (int i = 0; i < N; ++i) {
          double r[2], delta[2];
          int8_t sv = w->s[(size_t)(l - 1) * N + i];
          for (int sp = 0; sp < 2; ++sp) {
            int m = w->ne[sp];
            double sigma = sp == 0 ? 1.0 : -1.0;
            delta[sp] = exp(-2.0 * sigma * w->lambda * (double)sv) - 1.0;
            double a = 0.0;
            for (int p = 0; p < m; ++p) {
              double acc = 0.0;
              for (int q = 0; q < m; ++q) acc += w->Minv[sp][p * m + q] * X[sp][(size_t)i * m + q];
              a += PhiR[sp][(size_t)i * m + p] * acc;
            }
            r[sp] = 1.0 + delta[sp] * a;
          }
          double ratio = r[0] * r[1];
          double xr = orc_uniform(w->seed, w->wid, ORC_S_FLIP, sw, (uint32_t)(l - 1), (uint32_t)i);
          w->st.flip_attempts++;
          if (fabs(xr - fabs(ratio)) < 1e-9) w->st.near_ties++;
          if (xr < fabs(ratio)) {
            w->st.flip_accepts++;
            for (int sp = 0; sp < 2; ++sp) {
              int m = w->ne[sp];
              double *Mi = w->Minv[sp];
              /* Sherman-Morrison: Minv -= (delta/r) (Minv Phi_L[:,i]) (Phi_R[i,:] Minv) */
              for (int p = 0; p < m; ++p) {
                double acc = 0.0;
                for (int q = 0; q < m; ++q) acc += Mi[p * m + q] * X[sp][(size_t)i * m + q];
                u[p] = acc;
              }
              for (int q = 0; q < m; ++q) {
                double acc = 0.0;
                for (int p = 0; p < m; ++p) acc += PhiR[sp][(size_t)i * m + p] * Mi[p * m + q];
                wr[q] = acc;
              }
              double c = delta[sp] / r[sp];
              for (int p = 0; p < m; ++p)
                for (int q = 0; q < m; ++q) Mi[p * m + q] -= c * u[p] * wr[q];
              for (int p = 0; p < m; ++p) PhiR[sp][(size_t)i * m + p] *= 1.0 + delta[sp];
            }
            w->s[(size_t)(l - 1) * N + i] = (int8_t)(-sv);
            w->logw += log(fabs(ratio));
            if (ratio < 0.0) w->sign = -w->sign;
          }
        }
      }
      for (int sp = 0; sp < 2; ++sp) {
        ek_left(w, PhiR[sp], w->ne[sp]);
        ekinvT_left(w, X[sp], w->ne[sp]);
      }
    }
    /* end of block k: QR stabilisation, push (Q_k, V_k) */
    for (int sp = 0; sp < 2; ++sp) {
      int m = w->ne[sp];
      if (k < n && m > 0) {
        /* wrapped A_ii, compared with the fresh one at the next block start */
        for (int i = 0; i < N; ++i) {
          double acc = 0.0;
          for (int p = 0; p < m; ++p)
            for (int q = 0; q < m; ++q)
              acc += PhiR[sp][(size_t)i * m + p] * w->Minv[sp][p * m + q] * X[sp][(size_t)i * m + q];
          Aw[i] = acc;
        }
      }
      double *Q = w->RQ[sp] + (size_t)(k - 1) * N * m, *V = w->RV[sp] + (size_t)(k - 1) * m * m;
      qr_pos(PhiR[sp], N, m, Q, V);
      memcpy(PhiR[sp], Q, sizeof(double) * (size_t)N * m);
      if (k < n && m > 0) {
        const double *Xf = LS[sp] + (size_t)k * N * m;
        double *Mf = malloc(sizeof(double) * m * m), *Mfi = malloc(sizeof(double) * m * m);
        xty(Xf, PhiR[sp], N, m, Mf);
        double la; int sg;
        lu_inverse(Mf, m, Mfi, &la, &sg);
        for (int i = 0; i < N; ++i) {
          double acc = 0.0;
          for (int p = 0; p < m; ++p)
            for (int q = 0; q < m; ++q)
              acc += PhiR[sp][(size_t)i * m + p] * Mfi[p * m + q] * Xf[(size_t)i * m + q];
          double d = fabs(acc - Aw[i]);
          if (d > w->st.max_wrap_err) w->st.max_wrap_err = d;
        }
        free(Mf); free(Mfi);
      }
    }
  }
  /* tau = beta: M = P^T Q_n and the fresh weight */
  double la_tot = 0.0; int sg_tot = 1;
  for (int sp = 0; sp < 2; ++sp) {
    int m = w->ne[sp];
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < m; ++j) la_tot += log(w->RV[sp][(size_t)k * m * m + j * m + j]);
    double la; int sg;
    inverse_at_beta(w, sp, &la, &sg);
    la_tot += la; sg_tot *= sg;
  }
  w->stack_valid = 1;
  double drift = fabs(la_tot - w->logw);
  if (drift > w->st.logw_drift) w->st.logw_drift = drift;
  w->logw = la_tot; w->sign = sg_tot;
  if (n == 1 && do_measure) {
    for (int sp = 0; sp < 2; ++sp) {
      int m = w->ne[sp];
      fill_P(w, sp, X[sp]);
      build_A(N, m, w->RQ[sp], w->Minv[sp], X[sp], A[sp]);
    }
    measure_point(w, A, sg_tot);
  }
  free(Aw); free(u); free(wr);
  for (int sp = 0; sp < 2; ++sp) { free(LS[sp]); free(PhiR[sp]); free(X[sp]); free(M[sp]); free(A[sp]); }
  /* Fock-state phase: particle-hole swaps at tau = beta */
  if (!(w->flags & ORC_NO_FOCK)) {
    for (int sp = 0; sp < 2; ++sp) {
      int ne = w->ne[sp];
      if (ne == 0 || ne == N) continue;
      for (int mm = 0; mm < ne; ++mm) {
        int k = pick(orc_uniform(w->seed, w->wid, ORC_S_SWAP_K, sw, (uint32_t)sp, (uint32_t)mm), ne);
        int jn = pick(orc_uniform(w->seed, w->wid, ORC_S_SWAP_J, sw, (uint32_t)sp, (uint32_t)mm), N - ne);
        int j = nth_empty_site(w, sp, jn);
        swap_work x;
        swap_compute(w, sp, k, j, &x);
        double xr = orc_uniform(w->seed, w->wid, ORC_S_SWAP_ACC, sw, (uint32_t)sp, (uint32_t)mm);
        w->st.swap_attempts++;
        if (!x.zero && fabs(xr - exp(x.log_abs_r)) < 1e-9) w->st.near_ties++;
        if (!x.zero && xr < exp(x.log_abs_r)) {
          w->st.swap_accepts++;
          swap_commit(w, sp, &x);
          w->logw += x.log_abs_r;
          w->sign *= x.sign_r;
        }
        sw_free(&x);
      }
    }
  }
}

int orc_sweep(orc_walker *w, int32_t n_sweeps, int32_t do_measure) {
  if (!w || n_sweeps < 0) { set_err("bad argument"); return -1; }
  for (int t = 0; t < n_sweeps; ++t) one_sweep(w, do_measure);
  return 0;
}

int orc_log_weight(orc_walker *w, double *log_abs_w, int32_t *sign) {
  double la; int sg;
  fresh_weight(w, &la, &sg);
  *log_abs_w = la; *sign = sg;
  return 0;
}

int orc_tracked_weight(const orc_walker *w, double *log_abs_w, int32_t *sign) {
  *log_abs_w = w->logw; *sign = w->sign;
  return 0;
}

int orc_get_state(const orc_walker *w, int8_t *fields, int32_t *occ_up, int32_t *occ_dn, uint64_t *sweep_counter) {
  if (fields) memcpy(fields, w->s, (size_t)w->L * w->N);
  if (occ_up) for (int a = 0; a < w->ne[0]; ++a) occ_up[a] = w->occ[0][a];
  if (occ_dn) for (int a = 0; a < w->ne[1]; ++a) occ_dn[a] = w->occ[1][a];
  if (sweep_counter) *sweep_counter = w->sweep;
  return 0;
}

int orc_set_state(orc_walker *w, const int8_t *fields, const int32_t *occ_up, const int32_t *occ_dn, uint64_t sweep_counter) {
  for (int sp = 0; sp < 2; ++sp) {
    const int32_t *g = sp == 0 ? occ_up : occ_dn;
    if (!g) continue;
    char *used = calloc(w->N, 1);
    for (int a = 0; a < w->ne[sp]; ++a)
      if (g[a] < 0 || g[a] >= w->N || used[g[a]]) { free(used); set_err("bad occupation list"); return -1; }
      else used[g[a]] = 1;
    free(used);
  }
  if (fields)
    for (size_t t = 0; t < (size_t)w->L * w->N; ++t) w->s[t] = fields[t] > 0 ? 1 : -1;
  if (occ_up) for (int a = 0; a < w->ne[0]; ++a) w->occ[0][a] = occ_up[a];
  if (occ_dn) for (int a = 0; a < w->ne[1]; ++a) w->occ[1][a] = occ_dn[a];
  w->sweep = (uint32_t)sweep_counter;
  fresh_weight(w, &w->logw, &w->sign);
  return 0;
}

/* stabilised right state at boundary b: Q with B_b ... B_1 P = Q R */
static void right_state(const orc_walker *w, int sp, int b, double *Q) {
  int N = w->N, m = w->ne[sp];
  double *Phi = malloc(sizeof(double) * (size_t)N * (m ? m : 1));
  double *R = malloc(sizeof(double) * (m ? m * m : 1));
  fill_P(w, sp, Phi);
  for (int l = 1; l <= b; ++l) {
    diag_left(w, Phi, m, l, sp, 0);
    ek_left(w, Phi, m);
    if (l % w->nstab == 0 || l == b) { qr_pos(Phi, N, m, Q, R); memcpy(Phi, Q, sizeof(double) * (size_t)N * m); }
  }
  memcpy(Q, Phi, sizeof(double) * (size_t)N * m);
  free(Phi); free(R);
}
/* stabilised left state at boundary b: X (N x m) spanning (P^T B_L ... B_{b+1})^T */
static void left_state(const orc_walker *w, int sp, int b, double *X) {
  int N = w->N, m = w->ne[sp];
  double *Y = malloc(sizeof(double) * (size_t)N * (m ? m : 1));
  double *R = malloc(sizeof(double) * (m ? m * m : 1));
  fill_P(w, sp, Y);
  int cnt = 0;
  for (int l = w->L; l > b; --l) {
    ekT_left(w, Y, m);
    diag_left(w, Y, m, l, sp, 0);
    if (++cnt % w->nstab == 0 || l == b + 1) { qr_pos(Y, N, m, X, R); memcpy(Y, X, sizeof(double) * (size_t)N * m); }
  }
  memcpy(X, Y, sizeof(double) * (size_t)N * m);
  free(Y); free(R);
}

int orc_green(orc_walker *w, int32_t boundary, int32_t spin, double *G) {
  if (boundary < 0 || boundary > w->L || spin < 0 || spin > 1) { set_err("bad argument"); return -1; }
  int N = w->N, m = w->ne[spin];
  double *Q = malloc(sizeof(double) * (size_t)N * (m ? m : 1));
  double *X = malloc(sizeof(double) * (size_t)N * (m ? m : 1));
  double *M = malloc(sizeof(double) * (m ? m * m : 1)), *Mi = malloc(sizeof(double) * (m ? m * m : 1));
  double *A = malloc(sizeof(double) * (size_t)N * N);
  right_state(w, spin, boundary, Q);
  left_state(w, spin, boundary, X);
  xty(X, Q, N, m, M);
  double la; int sg;
  int rc = lu_inverse(M, m, Mi, &la, &sg);
  build_A(N, m, Q, Mi, X, A);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) G[(size_t)i * N + j] = (i == j ? 1.0 : 0.0) - A[(size_t)i * N + j];
  free(Q); free(X); free(M); free(Mi); free(A);
  if (rc) { set_err("singular P^T B P"); return -3; }
  return 0;
}

int orc_flip_ratio(orc_walker *w, int32_t slice, int32_t site, double *ratio) {
  if (slice < 0 || slice >= w->L || site < 0 || site >= w->N) { set_err("bad argument"); return -1; }
  int N = w->N, l = slice + 1;
  double r = 1.0;
  for (int sp = 0; sp < 2; ++sp) {
    int m = w->ne[sp];
    if (m == 0) continue;
    double *Q = malloc(sizeof(double) * (size_t)N * m), *X = malloc(sizeof(double) * (size_t)N * m);
    double *M = malloc(sizeof(double) * m * m), *Mi = malloc(sizeof(double) * m * m);
    right_state(w, sp, l - 1, Q);          /* B_{l-1} ... B_1 P */
    diag_left(w, Q, m, l, sp, 0);          /* D_l: the flip point */
    left_state(w, sp, l, X);               /* (P^T B_L ... B_{l+1})^T */
    ekT_left(w, X, m);                     /* (Phi_L E_K)^T */
    xty(X, Q, N, m, M);
    double la; int sg;
    lu_inverse(M, m, Mi, &la, &sg);
    double a = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q) a += Q[(size_t)site * m + p] * Mi[p * m + q] * X[(size_t)site * m + q];
    double sigma = sp == 0 ? 1.0 : -1.0;
    double delta = exp(-2.0 * sigma * w->lambda * (double)w->s[(size_t)slice * N + site]) - 1.0;
    r *= 1.0 + delta * a;
    free(Q); free(X); free(M); free(Mi);
  }
  *ratio = r;
  return 0;
}

static int check_swap(orc_walker *w, int spin, int k, int j) {
  if (spin < 0 || spin > 1) return -1;
  int ne = w->ne[spin];
  if (ne == 0 || ne == w->N || k < 0 || k >= ne || j < 0 || j >= w->N) return -1;
  for (int a = 0; a < ne; ++a) if (w->occ[spin][a] == j) return -1;
  return 0;
}

int orc_swap_ratio(orc_walker *w, int32_t spin, int32_t k_index, int32_t j_site, double *ratio) {
  if (check_swap(w, spin, k_index, j_site)) { set_err("bad swap"); return -1; }
  double la; int sg;
  fresh_weight(w, &la, &sg);
  swap_work x;
  swap_compute(w, spin, k_index, j_site, &x);
  *ratio = x.zero ? 0.0 : x.sign_r * exp(x.log_abs_r);
  sw_free(&x);
  return 0;
}

int orc_swap_commit(orc_walker *w, int32_t spin, int32_t k_index, int32_t j_site, double *ratio) {
  if (check_swap(w, spin, k_index, j_site)) { set_err("bad swap"); return -1; }
  if (!w->stack_valid) { double la; int sg; fresh_weight(w, &la, &sg); }
  swap_work x;
  swap_compute(w, spin, k_index, j_site, &x);
  *ratio = x.zero ? 0.0 : x.sign_r * exp(x.log_abs_r);
  if (!x.zero) {
    swap_commit(w, spin, &x);
    w->logw += x.log_abs_r;
    w->sign *= x.sign_r;
  }
  sw_free(&x);
  return x.zero ? -3 : 0;
}

int orc_right_stack(const orc_walker *w, int32_t spin, int32_t level, double *Q, double *V) {
  if (spin < 0 || spin > 1 || level < 0 || level >= w->nblk) { set_err("bad argument"); return -1; }
  int m = w->ne[spin];
  if (Q) memcpy(Q, w->RQ[spin] + (size_t)level * w->N * m, sizeof(double) * (size_t)w->N * m);
  if (V) memcpy(V, w->RV[spin] + (size_t)level * m * m, sizeof(double) * (size_t)m * m);
  return 0;
}

int orc_inverse(const orc_walker *w, int32_t spin, double *Minv) {
  int m = w->ne[spin];
  memcpy(Minv, w->Minv[spin], sizeof(double) * (size_t)m * m);
  return 0;
}

int64_t orc_obs_size(const orc_walker *w) { return w->nobs; }
int orc_measure(const orc_walker *w, double *out) { memcpy(out, w->obs, sizeof(double) * w->nobs); return 0; }
int orc_reset_measure(orc_walker *w) { memset(w->obs, 0, sizeof(double) * w->nobs); return 0; }
int orc_get_stats(const orc_walker *w, orc_stats *st) { *st = w->st; return 0; }

/* ======================================================================== */
/* Constrained-path (phaseless) LEC-QMC, SM Sec. VI.                         */
/*                                                                          */
/* Two-stage sampling: the outer chain draws Fock states eta with the       */
/* trial weight W_T(eta) = <eta| e^{-beta H_0} |eta> (the LEC-QMC chain of a */
/* walker with U = 0, driven by orc_sweep); for one eta the inner branching */
/* random walk estimates                                                    */
/*   R(eta) = E_s[ prod_sigma det(P^T B^sigma(s) P) ] / W_T(eta),            */
/* s uniform over the Ising fields (P(s) = 2^{-N L}), as the telescoping     */
/* product of overlap ratios O_T(tau_l) / O_T(tau_{l-1}) with the backward   */
/* trial state <psi(tau_l)| = <eta| e^{-(beta - tau_l) H_0}.                 */
/* H_0 is the one-body part (checkerboard hopping and onsite energies), so   */
/* B_l(s) = E_K D0 F_l(s), F_l(s) = diag(exp(sigma lambda s_{l,i})).          */
/* Across E_K D0 the overlap matrix X^T Phi is unchanged (the trial state    */
/* moves back by the same factor), so each slice's ratio is the product of   */
/* its site-by-site rank-1 ratios                                           */
/*   r_sigma(s) = 1 + (e^{sigma lambda s} - 1) [Phi (X^T Phi)^{-1} X^T]_ii,  */
/* updated sequentially (Sherman-Morrison) as the fields are drawn.          */
/* Phaseless constraint: a factor max(0, r) (the Hubbard fields are real, so */
/* the real part is the ratio itself); a walker whose factor is 0 is dead.   */
/* Stabilisation: the walker Phi = U_R D_R is replaced by U_R (thin QR) at   */
/* every block end and the trial state by the QR'd block boundary state U_L  */
/* of the H_0 left stack; the scales cancel in every ratio.                  */
/* Field sampling (mode):                                                    */
/*   ORC_CP_IMPORTANCE: s drawn with p(s) = P(s) max(0, r(s)) / N_i, weight  */
/*     times N_i = sum_s P(s) max(0, r(s)) (the walker-dependent, site by    */
/*     site sampling probability);                                          */
/*   ORC_CP_FREE: s drawn from P(s), weight times max(0, r(s)).              */
/* Population control (every pc_every slices, 0 = never): a comb over the   */
/* cumulative weights with one uniform draw; every copy carries the mean    */
/* weight, whose log is accumulated into the estimator.                     */
/* ======================================================================== */
struct orc_cp {
  orc_walker *tw;            /* U = 0 walker: tables, eta, H_0 left stack */
  double lambda;             /* Ising coupling of the interacting propagator */
  int nw, mode, pc_every, N, L;
  int ne[2];
  uint64_t seed;
  double *Phi[2];            /* [nw][N][ne] */
  double *Minv[2];           /* [nw][ne][ne] */
  double *logw;              /* [nw], -INFINITY = dead */
  double *logq;              /* [nw] sum of log p(s) of the drawn fields (importance mode) */
  int8_t *s;                 /* [nw][L][N] drawn field path */
  double log_pc;             /* sum of log(mean weight) over the population controls */
  int64_t cuts;              /* site updates at which a walker died */
};

static void cp_free_walkers(orc_cp *c) {
  for (int sp = 0; sp < 2; ++sp) { free(c->Phi[sp]); free(c->Minv[sp]); c->Phi[sp] = c->Minv[sp] = NULL; }
  free(c->logw); free(c->logq); free(c->s);
  c->logw = c->logq = NULL; c->s = NULL;
}

orc_cp *orc_cp_create(const orc_lattice *lat, const orc_params *par, const int32_t *occ_up,
                      const int32_t *occ_dn, int32_t n_walkers, int32_t mode, int32_t pc_every) {
  if (!lat || !par || !occ_up || !occ_dn) { set_err("null argument"); return NULL; }
  if (n_walkers <= 0 || (mode != ORC_CP_IMPORTANCE && mode != ORC_CP_FREE) || pc_every < 0) {
    set_err("bad walker count, mode or control interval"); return NULL;
  }
  orc_params p0 = *par;
  p0.U = 0.0;
  p0.flags = ORC_NO_FLIPS | ORC_NO_FOCK;
  orc_walker *tw = orc_create(lat, &p0, NULL, occ_up, occ_dn);
  if (!tw) return NULL;
  orc_cp *c = calloc(1, sizeof *c);
  c->tw = tw;
  c->lambda = acosh(exp(par->dtau * par->U / 2.0));
  c->nw = n_walkers; c->mode = mode; c->pc_every = pc_every;
  c->N = tw->N; c->L = tw->L; c->ne[0] = tw->ne[0]; c->ne[1] = tw->ne[1];
  c->seed = par->seed;
  for (int sp = 0; sp < 2; ++sp) {
    size_t m = c->ne[sp] ? (size_t)c->ne[sp] : 1;
    c->Phi[sp] = malloc(sizeof(double) * (size_t)n_walkers * c->N * m);
    c->Minv[sp] = malloc(sizeof(double) * (size_t)n_walkers * m * m);
  }
  c->logw = malloc(sizeof(double) * n_walkers);
  c->logq = malloc(sizeof(double) * n_walkers);
  c->s = malloc((size_t)n_walkers * c->L * c->N);
  return c;
}

void orc_cp_destroy(orc_cp *c) {
  if (!c) return;
  cp_free_walkers(c);
  orc_destroy(c->tw);
  free(c);
}

/* fresh (X^T Phi)^{-1} of walker a, spin sp */
static void cp_fresh_inverse(orc_cp *c, int a, int sp, const double *X) {
  int N = c->N, m = c->ne[sp];
  if (m == 0) return;
  double *M = malloc(sizeof(double) * m * m);
  xty(X, c->Phi[sp] + (size_t)a * N * m, N, m, M);
  double la; int sg;
  lu_inverse(M, m, c->Minv[sp] + (size_t)a * m * m, &la, &sg);
  free(M);
}

/* comb: nw copies chosen at the positions (j + xi) W / nw of the cumulative
 * weights; every copy carries weight W / nw (log accumulated in log_pc) */
static void cp_comb(orc_cp *c, double xi) {
  int nw = c->nw, N = c->N, L = c->L;
  double mx = -INFINITY;
  for (int a = 0; a < nw; ++a) if (c->logw[a] > mx) mx = c->logw[a];
  if (mx == -INFINITY) return;  /* every walker dead: nothing to resample */
  double *cum = malloc(sizeof(double) * nw);
  double W = 0.0;
  for (int a = 0; a < nw; ++a) { W += exp(c->logw[a] - mx); cum[a] = W; }
  int *pick_of = malloc(sizeof(int) * nw);
  int a = 0;
  for (int j = 0; j < nw; ++j) {
    double t = ((double)j + xi) * W / (double)nw;
    while (a < nw - 1 && cum[a] <= t) ++a;
    /* rounding can carry t onto a dead walker's empty interval: take the
     * nearest live walker instead */
    int b = a;
    while (b > 0 && c->logw[b] == -INFINITY) --b;
    while (b < nw - 1 && c->logw[b] == -INFINITY) ++b;
    pick_of[j] = b;
  }
  double *Phi[2], *Minv[2];
  for (int sp = 0; sp < 2; ++sp) {
    size_t m = c->ne[sp] ? (size_t)c->ne[sp] : 1;
    Phi[sp] = malloc(sizeof(double) * (size_t)nw * N * m);
    Minv[sp] = malloc(sizeof(double) * (size_t)nw * m * m);
    for (int j = 0; j < nw; ++j) {
      memcpy(Phi[sp] + (size_t)j * N * m, c->Phi[sp] + (size_t)pick_of[j] * N * m, sizeof(double) * N * m);
      memcpy(Minv[sp] + (size_t)j * m * m, c->Minv[sp] + (size_t)pick_of[j] * m * m, sizeof(double) * m * m);
    }
    free(c->Phi[sp]); free(c->Minv[sp]);
    c->Phi[sp] = Phi[sp]; c->Minv[sp] = Minv[sp];
  }
  int8_t *s = malloc((size_t)nw * L * N);
  double *lq = malloc(sizeof(double) * nw);
  for (int j = 0; j < nw; ++j) {
    memcpy(s + (size_t)j * L * N, c->s + (size_t)pick_of[j] * L * N, (size_t)L * N);
    lq[j] = c->logq[pick_of[j]];
  }
  free(c->s); c->s = s;
  free(c->logq); c->logq = lq;
  c->log_pc += mx + log(W / (double)nw);
  for (int j = 0; j < nw; ++j) c->logw[j] = 0.0;
  free(cum); free(pick_of);
}

/* one site update of walker a at slice l, site i (fields drawn here) */
static void cp_site(orc_cp *c, int a, int l, int i, uint32_t tag, double *const X[2], double *u, double *v) {
  int N = c->N;
  double g[2];
  for (int sp = 0; sp < 2; ++sp) {
    int m = c->ne[sp];
    const double *Mi = c->Minv[sp] + (size_t)a * m * m;
    const double *ph = c->Phi[sp] + ((size_t)a * N + i) * m;
    double acc = 0.0;
    for (int p = 0; p < m; ++p) {
      double t = 0.0;
      for (int q = 0; q < m; ++q) t += Mi[p * m + q] * X[sp][(size_t)i * m + q];
      acc += ph[p] * t;
    }
    g[sp] = acc;   /* [Phi (X^T Phi)^{-1} X^T]_ii */
  }
  double f[2];  /* max(0, r(s)) for s = +1, -1; r = product over spins */
  for (int t = 0; t < 2; ++t) {
    double sv = t == 0 ? 1.0 : -1.0;
    double prod = 1.0;
    for (int sp = 0; sp < 2; ++sp) {
      double sigma = sp == 0 ? 1.0 : -1.0;
      prod *= 1.0 + (exp(sigma * c->lambda * sv) - 1.0) * g[sp];
    }
    f[t] = prod > 0.0 ? prod : 0.0;
  }
  double x = orc_uniform(c->seed, (uint64_t)a, ORC_S_CP_FIELD, tag, (uint32_t)(l - 1), (uint32_t)i);
  int t;
  double factor;
  if (c->mode == ORC_CP_IMPORTANCE) {
    double Ni = 0.5 * f[0] + 0.5 * f[1];
    if (Ni == 0.0) { c->logw[a] = -INFINITY; c->cuts++; return; }
    double p_plus = 0.5 * f[0] / Ni;
    t = x < p_plus ? 0 : 1;
    factor = Ni;
    c->logq[a] += log(t == 0 ? p_plus : 1.0 - p_plus);
  } else {
    t = x < 0.5 ? 0 : 1;
    factor = f[t];
    if (factor == 0.0) { c->logw[a] = -INFINITY; c->cuts++; return; }
  }
  double sv = t == 0 ? 1.0 : -1.0;
  c->s[((size_t)a * c->L + (l - 1)) * N + i] = (int8_t)(t == 0 ? 1 : -1);
  c->logw[a] += log(factor);
  /* apply F_i(s) to the walker: Phi[i,:] *= 1 + delta, Sherman-Morrison on (X^T Phi)^{-1} */
  for (int sp = 0; sp < 2; ++sp) {
    int m = c->ne[sp];
    if (m == 0) continue;
    double sigma = sp == 0 ? 1.0 : -1.0;
    double delta = exp(sigma * c->lambda * sv) - 1.0;
    double rs = 1.0 + delta * g[sp];
    double *Mi = c->Minv[sp] + (size_t)a * m * m;
    double *ph = c->Phi[sp] + ((size_t)a * N + i) * m;
    for (int p = 0; p < m; ++p) {
      double acc = 0.0;
      for (int q = 0; q < m; ++q) acc += Mi[p * m + q] * X[sp][(size_t)i * m + q];
      u[p] = acc;
    }
    for (int q = 0; q < m; ++q) {
      double acc = 0.0;
      for (int p = 0; p < m; ++p) acc += ph[p] * Mi[p * m + q];
      v[q] = acc;
    }
    double cc = delta / rs;
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q) Mi[p * m + q] -= cc * u[p] * v[q];
    for (int p = 0; p < m; ++p) ph[p] *= 1.0 + delta;
  }
}

int orc_cp_run(orc_cp *c, uint32_t tag, double *log_r) {
  if (!c || !log_r) { set_err("null argument"); return -1; }
  orc_walker *tw = c->tw;
  int N = c->N, n = tw->nblk, nw = c->nw;
  double *LS[2], *X[2];
  for (int sp = 0; sp < 2; ++sp) {
    size_t m = c->ne[sp] ? (size_t)c->ne[sp] : 1;
    LS[sp] = left_stack(tw, sp);         /* H_0 left stack (lambda = 0) */
    X[sp] = malloc(sizeof(double) * N * m);
    for (int a = 0; a < nw; ++a) fill_P(tw, sp, c->Phi[sp] + (size_t)a * N * m);
  }
  for (int a = 0; a < nw; ++a) { c->logw[a] = 0.0; c->logq[a] = 0.0; }
  memset(c->s, 0, (size_t)nw * c->L * N);
  c->log_pc = 0.0;
  c->cuts = 0;
  int mmax = c->ne[0] > c->ne[1] ? c->ne[0] : c->ne[1];
  double *u = malloc(sizeof(double) * (mmax + 1)), *v = malloc(sizeof(double) * (mmax + 1));
  for (int k = 1; k <= n; ++k) {
    for (int sp = 0; sp < 2; ++sp) {
      int m = c->ne[sp];
      memcpy(X[sp], LS[sp] + (size_t)(k - 1) * N * m, sizeof(double) * (size_t)N * m);
      for (int a = 0; a < nw; ++a)
        if (c->logw[a] > -INFINITY) cp_fresh_inverse(c, a, sp, X[sp]);
    }
    for (int l = block_first(tw, k); l <= block_last(tw, k); ++l) {
      /* D0 on the walkers, D0^{-1} on the trial state: the flip point of slice l */
      for (int sp = 0; sp < 2; ++sp) {
        int m = c->ne[sp];
        diag_left(tw, X[sp], m, l, sp, 1);
        for (int a = 0; a < nw; ++a)
          if (c->logw[a] > -INFINITY) diag_left(tw, c->Phi[sp] + (size_t)a * N * m, m, l, sp, 0);
      }
      for (int a = 0; a < nw; ++a)
        for (int i = 0; i < N && c->logw[a] > -INFINITY; ++i) cp_site(c, a, l, i, tag, X, u, v);
      for (int sp = 0; sp < 2; ++sp) {
        int m = c->ne[sp];
        ekinvT_left(tw, X[sp], m);
        for (int a = 0; a < nw; ++a)
          if (c->logw[a] > -INFINITY) ek_left(tw, c->Phi[sp] + (size_t)a * N * m, m);
      }
      if (l == block_last(tw, k))
        for (int sp = 0; sp < 2; ++sp) {
          int m = c->ne[sp];
          if (m == 0) continue;
          double *Q = malloc(sizeof(double) * (size_t)N * m), *R = malloc(sizeof(double) * m * m);
          for (int a = 0; a < nw; ++a) {
            if (c->logw[a] == -INFINITY) continue;
            double *ph = c->Phi[sp] + (size_t)a * N * m;
            qr_pos(ph, N, m, Q, R);
            memcpy(ph, Q, sizeof(double) * (size_t)N * m);
          }
          free(Q); free(R);
        }
      if (c->pc_every > 0 && l % c->pc_every == 0 && l < c->L) {
        cp_comb(c, orc_uniform(c->seed, 0, ORC_S_CP_COMB, tag, (uint32_t)(l - 1), 0));
        /* the copies' inverses are copied with them; mid-block they stay valid */
      }
    }
  }
  double mx = -INFINITY;
  for (int a = 0; a < nw; ++a) if (c->logw[a] > mx) mx = c->logw[a];
  if (mx == -INFINITY) {
    *log_r = -INFINITY;
  } else {
    double W = 0.0;
    for (int a = 0; a < nw; ++a) W += exp(c->logw[a] - mx);
    *log_r = c->log_pc + mx + log(W / (double)nw);
  }
  free(u); free(v);
  for (int sp = 0; sp < 2; ++sp) { free(LS[sp]); free(X[sp]); }
  return 0;
}

int orc_cp_walker(const orc_cp *c, int32_t a, double *log_w, double *log_q, int8_t *fields) {
  if (!c || a < 0 || a >= c->nw) { set_err("bad walker index"); return -1; }
  if (log_w) *log_w = c->logw[a];
  if (log_q) *log_q = c->logq[a];
  if (fields) memcpy(fields, c->s + (size_t)a * c->L * c->N, (size_t)c->L * c->N);
  return 0;
}

int orc_cp_stats(const orc_cp *c, double *log_pc, int64_t *cuts, int32_t *alive) {
  if (!c) { set_err("null argument"); return -1; }
  if (log_pc) *log_pc = c->log_pc;
  if (cuts) *cuts = c->cuts;
  if (alive) {
    int n = 0;
    for (int a = 0; a < c->nw; ++a) n += c->logw[a] > -INFINITY;
    *alive = n;
  }
  return 0;
}
