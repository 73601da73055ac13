// Host side of the C ABI declared in include/lecqmc.h: validation, model
// tables, device-memory layout of a walker, and kernel orchestration.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/lecqmc.h"
#include "lecqmc_internal.h"

using namespace lecqmc;

static thread_local char g_err[512];

static int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(LECQMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Descriptor staging of lecqmc_sweep_batch_static: one array in each
// device's memory, held until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (lecqmc_ctx_create), and is kept in
// g_scratch_addr.
constexpr int kStaticMaxWalkers = LECQMC_STATIC_MAX_WALKERS;
static __device__ __align__(256) unsigned char scratch[kStaticMaxWalkers * sizeof(WalkerDesc)];
static std::mutex g_scratch_mu;
static std::map<int, WalkerDesc *> g_scratch_addr;

struct lecqmc_ctx {
  int device;
  WalkerDesc *scratch_desc;   // this device's copy of scratch (device address)
  hipStream_t stream;
  bool own_stream;
  size_t budget, used;
  WalkerDesc *d_batch;
  int batch_cap;
  // earlier descriptor arrays, freed with the context: freeing device memory
  // waits for the whole device, which would stall other contexts' work
  std::vector<WalkerDesc *> old_batches;
  int live_walkers;
  bool timing;
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // autotuned flip-chain shapes by (N, Ne_up, Ne_dn, precision); new walkers
  // of a tuned key start with its shape
  std::map<std::tuple<int, int, int, int>, std::pair<int, int>> tuned;
};

static hipEvent_t take_event(lecqmc_ctx *c) {
  if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Host <-> device transfers and clears run on the context's own stream and
// wait for that stream alone: work on the shared default stream can queue
// behind other contexts' kernels (streams share the hardware queues).
static hipError_t xfer(lecqmc_ctx *c, void *dst, const void *src, size_t n, hipMemcpyKind kind) {
  if (n == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dst, src, n, kind, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}
static hipError_t zero(lecqmc_ctx *c, void *dst, size_t n) {
  if (n == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(dst, 0, n, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

// launch one phase, bracketed by events when timing is on
template <typename F>
static hipError_t timed(lecqmc_ctx *c, int phase, F launch) {
  if (!c->timing) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  hipError_t e = hipEventRecord(a, c->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  c->recs.push_back({phase, a, b});
  return e;
}

struct lecqmc_walker {
  lecqmc_ctx *ctx;
  WalkerDesc h;          // descriptor with device pointers
  WalkerDesc *d_desc;    // device copy
  void *dmem;
  size_t bytes;
  int N, L, nblk, ne[2], mmax, nobs;
  int batches;           // live lecqmc_batch objects that hold this walker
};

extern "C" const char *lecqmc_last_error(void) { return g_err; }

// Flip-chain shape of a walker: the register tile T (the Ne x Ne inverse in
// registers for Ne <= 8T), T = 0 (the inverse in memory, site by site) or
// kDelayed (the delayed chunk update), and the sites per staged chunk.
// Defaults by Ne, from measurements of the forward pass; lecqmc_autotune
// replaces them by timed choices.  Every shape samples the same chain; the
// shape changes only the rounding of the ratios.
static bool shape_valid(int ne0, int ne1, int tile, int chunk);
static void shape_default(int ne0, int ne1, int *tile, int *chunk) {
  const int mmax = std::max(1, std::max(ne0, ne1));
  *tile = mmax <= 8 ? 1 : mmax <= 16 ? 2 : mmax <= 32 ? 4 : mmax <= kMfmaMaxNe ? kMfma : kDelayed;
  *chunk = mmax <= 16 ? 32 : mmax <= 32 ? 16 : *tile == kMfma ? kMS : 8;
  if (*tile == kMfma && !shape_valid(ne0, ne1, *tile, *chunk)) {
    *tile = kDelayed;
    *chunk = 8;
  }
  if (*tile == kDelayed && !shape_valid(ne0, ne1, *tile, *chunk)) *chunk = 4;
}
// row stride of the staged chunk rows: 8T for a register tile; Ne, or the
// next odd number for the delayed chain (its threads read rows side by side)
static int shape_xld(int mmax, int tile) {
  return (tile == kDelayed || tile == kMfma) ? (mmax | 1) : tile > 0 ? 8 * tile : mmax;
}
// LDS doubles of a shape's chunk matrices (0 for the site-by-site chains)
// (the matrix-core chain needs only G and Z in LDS: U, W move to device
// memory when the launch has no room for them)
static int shape_dgn(int ne0, int ne1, int tile, bool full = false) {
  return tile == kDelayed ? 4 * kDS * kDS : tile == kMfma ? (full ? mfma_lds_doubles(ne0, ne1) : mfma_lds_small()) : 0;
}
static bool shape_valid(int ne0, int ne1, int tile, int chunk) {
  const int mmax = std::max(1, std::max(ne0, ne1));
  if (!(tile == 0 || tile == 1 || tile == 2 || tile == 4 || tile == kDelayed || tile == kMfma)) return false;
  if (tile > 0 && tile != kDelayed && tile != kMfma && mmax > 8 * tile) return false;
  if (!(chunk == 4 || chunk == 8 || chunk == 16 || chunk == 32)) return false;
  if (tile == kDelayed && chunk > 16) return false;   // the delayed chain's registers hold 16 sites
  if (tile == kMfma && (chunk != kMS || mmax > kMfmaMaxNe)) return false;   // one 16-wide tile per chunk
  // both staging buffers (streamed walker) must fit next to the fixed layout,
  // with the Ne x Ne work matrices moved to device memory if need be (the
  // launch planner does that when they do not fit)
  const LdsPlan p{mmax, 0, 1, 0, 4 * chunk * shape_xld(mmax, tile), chunk, 1, shape_dgn(ne0, ne1, tile)};
  return lds_bytes(p) <= kLdsLimit;
}
static void shape_apply(WalkerDesc &h, int tile, int chunk) {
  h.tile = tile;
  h.chunk = chunk;
  h.xld = shape_xld(h.mmax, tile);
}

// LDS plan per launch: the fixed layout for the largest Ne and chunk of the
// launch, then room for resident Slater blocks (then the compact bond
// tables).  When the largest walker's blocks do not fit, the room is sized
// for the largest that do; the others stream theirs.
struct LaunchCfg {
  LdsPlan fwd, left, fock, meas;
  LdsPlan fresh;  // FP64 right chain of the fresh weight (all walkers)
  int slots;
  int mixed;      // FP32 storage in the sweep phases
  int tile;       // chain shape shared by all walkers, -1 if they differ
  bool fits;      // the launch's fixed LDS part fits (always for one walker)
};

static LdsPlan plan_for(LdsPlan p, const std::vector<long> &needs, int bond_need, bool staged_if_streamed) {
  long mx = 0;
  for (long v : needs) mx = std::max(mx, v);
  p.phi_elems = (int)mx;
  p.stage_ps = 0;
  p.bond_words = 0;
  if (mx <= 0 || lds_bytes(p) > kLdsLimit) {
    p.phi_elems = 0;
    p.stage_ps = staged_if_streamed ? 1 : 0;
    const size_t base = lds_bytes(p);
    const long cap = base < kLdsLimit ? (long)((kLdsLimit - base) / sizeof(double)) : 0;
    long best = 0;
    for (long v : needs)
      if (v <= cap) best = std::max(best, v);
    p.phi_elems = (int)best;
  }
  if (bond_need > 0) {
    p.bond_words = bond_need;
    if (lds_bytes(p) > kLdsLimit) p.bond_words = 0;
  }
  return p;
}

// Walkers of one launch share a precision (the sweep launchers group them).
// Resident blocks are counted in doubles: FP32 storage needs half of them.
static LaunchCfg launch_cfg(lecqmc_walker *const *ws, int n) {
  int mm = 1, bonds = 0, slots = 1, xs = 0, smax = 0, tile = n > 0 ? ws[0]->h.tile : 0, dgn = 0, dgn_min = 0;
  std::vector<long> fwd, left, fock, fresh;
  bool compact = true;
  const int mixed = n > 0 ? ws[0]->h.mixed : 0;
  const int eb = mixed ? (int)sizeof(float) : (int)sizeof(double);
  for (int t = 0; t < n; ++t) {
    const lecqmc_walker *w = ws[t];
    mm = std::max(mm, w->mmax);
    xs = std::max(xs, 4 * w->h.chunk * w->h.xld);
    smax = std::max(smax, w->h.chunk);
    fwd.push_back(phi_doubles((long)w->N * (w->ne[0] + w->ne[1]), eb));
    left.push_back(phi_doubles((long)w->N * std::max(w->ne[0], w->ne[1]), eb));
    fock.push_back(phi_doubles((long)w->N, eb));
    fresh.push_back((long)w->N * std::max(w->ne[0], w->ne[1]));
    if (w->h.ncoef == 0) compact = false;
    bonds = std::max(bonds, w->h.bond_words);
    slots = std::max(slots, w->nblk - 1);
    if (w->h.tile != tile) tile = -1;
    dgn = std::max(dgn, shape_dgn(w->ne[0], w->ne[1], w->h.tile, true));
    dgn_min = std::max(dgn_min, shape_dgn(w->ne[0], w->ne[1], w->h.tile, false));
  }
  if (!compact) bonds = 0;
  // The fixed part of the plan takes each region's largest size over the
  // walkers; when the Ne x Ne work matrices do not fit next to the rest, they
  // move to the walkers' device memory (same arithmetic, other memory).
  // Placement of the Ne x Ne work matrices per launch kind: the first of all
  // four in LDS, the two inverses in LDS, none -- the forward pass also
  // holds the chain staging, the other phases do not
  auto place = [&](LdsPlan worst) {
    worst.gm = 0;
    if (mm <= kLdsNe && lds_bytes(worst) <= kLdsLimit) return 0;
    worst.gm = 2;
    return lds_bytes(worst) <= kLdsLimit ? 2 : 1;
  };
  // the matrix-core chain's U and W stay in LDS only when the launch has
  // room for them next to everything else (staged right rows included)
  if (dgn > dgn_min && lds_bytes(LdsPlan{mm, 0, 1, 0, xs, smax, 1, dgn}) > kLdsLimit) dgn = dgn_min;
  const int gmf = place(LdsPlan{mm, 0, 1, 0, xs, smax, 0, dgn});
  const int gm = place(LdsPlan{mm, 0, 0, 0, 0, 0, 0, 0});
  if (gm) slots = 1;   // one estimator workgroup per walker: its work matrices are one per walker
  // the Fock phase keeps at least its Hessenberg work matrix in LDS when the
  // others have to go (its Givens chain reads a row of it per step)
  int gmk = gm;
  if (gm == 1 && lds_bytes(LdsPlan{mm, 0, 0, 0, 0, 0, 3, 0}) + sizeof(double) * std::max(64, mm) <= kLdsLimit) gmk = 3;
  const LdsPlan base{mm, 0, 0, 0, 0, 0, gm, 0}, fbase{mm, 0, 0, 0, xs, smax, gmf, dgn},
      kbase{mm, 0, 0, 0, 0, 0, gmk, 0};
  LdsPlan fw = fbase;
  fw.stage_ps = 1;
  return {plan_for(fbase, fwd, bonds, true), plan_for(base, left, bonds, false), plan_for(kbase, fock, bonds, false),
          base,                              plan_for(base, fresh, bonds, false), slots,
          mixed,                             tile,
          lds_bytes(fw) <= kLdsLimit};
}

// ---------------------------------------------------------------------------
// validation and memory plan
// ---------------------------------------------------------------------------
static int validate(const lecqmc_lattice *lat, const lecqmc_params *par, int *L_out) {
  if (!lat || !par) return fail(LECQMC_EINVAL, "null lattice or params");
  const int N = lat->n_sites;
  if (N <= 0 || lat->n_bonds < 0 || lat->n_colors < 0 || (lat->n_bonds > 0 && lat->n_colors <= 0))
    return fail(LECQMC_EINVAL, "bad lattice sizes");
  if (lat->n_bonds > 0 && (!lat->bond_i || !lat->bond_j || !lat->bond_color || !lat->bond_h))
    return fail(LECQMC_EINVAL, "missing bond arrays");
  if (par->n_up < 0 || par->n_up > N || par->n_dn < 0 || par->n_dn > N)
    return fail(LECQMC_EINVAL, "particle number out of [0, n_sites]");
  if (par->n_up > LECQMC_MAX_NE || par->n_dn > LECQMC_MAX_NE)
    return fail(LECQMC_EINVAL, "particle number per spin above %d", LECQMC_MAX_NE);
  if (par->n_stab <= 0) return fail(LECQMC_EINVAL, "n_stab must be >= 1");
  if (!(par->dtau > 0.0) || !(par->beta > 0.0)) return fail(LECQMC_EINVAL, "beta and dtau must be > 0");
  if (!(par->U >= 0.0)) return fail(LECQMC_EINVAL, "U must be >= 0 (spin-channel decoupling)");
  if (par->precision != LECQMC_FP64 && par->precision != LECQMC_MIXED)
    return fail(LECQMC_EINVAL, "unsupported precision %d", par->precision);
  const double Lf = par->beta / par->dtau;
  const long L = lround(Lf);
  if (L <= 0 || fabs(Lf - (double)L) > 1e-9 * (Lf > 1 ? Lf : 1)) return fail(LECQMC_EINVAL, "beta/dtau not integral");
  if ((double)L * N > 2.0e9) return fail(LECQMC_EINVAL, "field array too large");
  std::vector<int> seen(N, -1);
  for (int b = 0; b < lat->n_bonds; ++b) {
    const int i = lat->bond_i[b], j = lat->bond_j[b], c = lat->bond_color[b];
    if (i < 0 || i >= N || j < 0 || j >= N || i == j || c < 0 || c >= lat->n_colors)
      return fail(LECQMC_EINVAL, "bad bond %d", b);
  }
  for (int c = 0; c < lat->n_colors; ++c)
    for (int b = 0; b < lat->n_bonds; ++b) {
      if (lat->bond_color[b] != c) continue;
      const int i = lat->bond_i[b], j = lat->bond_j[b];
      if (seen[i] == c || seen[j] == c) return fail(LECQMC_EINVAL, "colour %d has a shared site", c);
      seen[i] = c;
      seen[j] = c;
    }
  const int ns = (lat->sublattice && lat->n_sublattices > 0) ? lat->n_sublattices : 1;
  if (ns > 8) return fail(LECQMC_EINVAL, "at most 8 sublattices");
  if (lat->sublattice)
    for (int i = 0; i < N; ++i)
      if (lat->sublattice[i] < 0 || lat->sublattice[i] >= ns) return fail(LECQMC_EINVAL, "bad sublattice index");
  *L_out = (int)L;
  return 0;
}

struct Plan {
  size_t off_sc, off_desc, off_s, off_occ[2], off_LS[2], off_LX[2], off_RQ[2], off_RV[2], off_Minv[2], off_PhiR[2], off_X[2],
      off_T[2], off_Aw[2], off_mpart, off_mscr, off_fq, off_fw, off_fVp, off_fgc, off_fgs, off_fv, off_frho, off_fmark, off_obs,
      off_dbg, off_col, off_bi, off_bj, off_bdiag, off_boff, off_bh, off_epsf, off_eps, off_sub, off_bij, off_bci,
      off_coef, off_bigm, off_dch;
  size_t mscr_stride;
  size_t total;
};

// per-boundary measurement scratch: T (2 N mmax), diagonals (2 N), all-pair A (2 N^2 if N <= 64)
static size_t meas_stride(int N, int mmax) {
  return 2 * (size_t)N * mmax + 2 * (size_t)N + (N <= 64 ? 2 * (size_t)N * N : 0);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int obs_count(int N, int ns) { return 8 + 2 * ns * ns + (N <= 64 ? 2 * N * N + 2 * N : 0); }

static Plan make_plan(int N, int L, int nstab, int ne0, int ne1, int nbonds, int ncol, int ns, int mixed) {
  Plan p;
  const int nb = (L + nstab - 1) / nstab;
  const int mmax = std::max(1, std::max(ne0, ne1));
  const int ne[2] = {ne0, ne1};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + (bytes ? bytes : 8)); return r; };
  p.off_sc = take(sizeof(Scalars));
  p.off_desc = take(sizeof(WalkerDesc));
  p.off_s = take((size_t)L * N);
  for (int s = 0; s < 2; ++s) p.off_occ[s] = take(sizeof(int) * (size_t)N);
  for (int s = 0; s < 2; ++s) {
    const size_t blk = (size_t)N * ne[s] * sizeof(double);
    p.off_LS[s] = take(blk * (nb + 1));
    p.off_LX[s] = take((size_t)N * ne[s] * (mixed ? sizeof(float) : sizeof(double)) * L);
    p.off_RQ[s] = take(blk * nb);
    p.off_RV[s] = take(sizeof(double) * (size_t)ne[s] * ne[s] * nb);
    p.off_Minv[s] = take(sizeof(double) * (size_t)ne[s] * ne[s]);
    p.off_PhiR[s] = take(blk);
    p.off_X[s] = take(blk);
    p.off_T[s] = take(blk);
    p.off_Aw[s] = take(sizeof(double) * (size_t)nb * N);
  }
  // measurement records and scratch, one per interior boundary (or tau = beta)
  const size_t slots = nb > 1 ? nb - 1 : 1;
  p.off_mpart = take(sizeof(double) * slots * (obs_count(N, ns) + 1));
  p.mscr_stride = meas_stride(N, mmax);
  p.off_mscr = take(sizeof(double) * slots * p.mscr_stride);
  // Fock-phase scratch, one copy per spin (the two spins run concurrently)
  p.off_fq = take(sizeof(double) * 2 * (size_t)nb * N);
  p.off_fw = take(sizeof(double) * 2 * (size_t)N);
  p.off_fVp = take(sizeof(double) * 2 * (size_t)nb * mmax * mmax);
  p.off_fgc = take(sizeof(double) * 2 * (size_t)nb * mmax);
  p.off_fgs = take(sizeof(double) * 2 * (size_t)nb * mmax);
  p.off_fv = take(sizeof(double) * 2 * (size_t)nb * mmax);
  p.off_frho = take(sizeof(double) * 2 * nb);
  p.off_fmark = take(sizeof(int) * 2 * (size_t)N);
  p.off_obs = take(sizeof(double) * obs_count(N, ns));
  p.off_dbg = take(sizeof(double) * (N <= 64 ? std::max(8, 2 * N * N) : 8));
  p.off_col = take(sizeof(int) * (ncol + 1));
  p.off_bi = take(sizeof(int) * nbonds);
  p.off_bj = take(sizeof(int) * nbonds);
  p.off_bdiag = take(sizeof(double) * nbonds);
  p.off_boff = take(sizeof(double) * nbonds);
  p.off_bh = take(sizeof(double) * nbonds);
  p.off_epsf = take(sizeof(double) * N);
  p.off_eps = take(sizeof(double) * N);
  p.off_sub = take(sizeof(int) * N);
  p.off_bij = take(sizeof(int) * nbonds);
  p.off_bci = take(nbonds);
  p.off_coef = take(sizeof(double) * 2 * kMaxCoef);
  p.off_bigm = take(sizeof(double) * 8 * (size_t)mmax * mmax);
  p.off_dch = take(sizeof(double) * (8 * (size_t)mmax * kDS + 4 * kDS * kDS));
  p.total = o;
  return p;
}

extern "C" size_t lecqmc_footprint_bytes(const lecqmc_lattice *lat, const lecqmc_params *par) {
  int L = 0;
  if (validate(lat, par, &L)) return 0;
  const int ns = (lat->sublattice && lat->n_sublattices > 0) ? lat->n_sublattices : 1;
  return make_plan(lat->n_sites, L, par->n_stab, par->n_up, par->n_dn, lat->n_bonds, lat->n_colors, ns,
                   par->precision == LECQMC_MIXED)
      .total;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int lecqmc_ctx_create(int device, void *stream, size_t budget, lecqmc_ctx **out) {
  if (!out) return fail(LECQMC_EINVAL, "null out");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(LECQMC_EINVAL, "device %d not present (%d devices)", device, ndev);
  HIPCHK(hipSetDevice(device));
  WalkerDesc *sd = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(LECQMC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      it = g_scratch_addr.emplace(device, (WalkerDesc *)p).first;
    }
    sd = it->second;
  }
  lecqmc_ctx *c = new lecqmc_ctx();
  c->device = device;
  c->scratch_desc = sd;
  c->budget = budget;
  c->used = 0;
  c->d_batch = nullptr;
  c->batch_cap = 0;
  c->timing = false;
  c->live_walkers = 0;
  if (stream) {
    c->stream = (hipStream_t)stream;
    c->own_stream = false;
  } else {
    // non-blocking: the library's synchronous host copies (legacy default
    // stream) then do not wait for kernels of other contexts' streams
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete c; return fail(LECQMC_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)); }
    c->own_stream = true;
  }
  *out = c;
  return 0;
}

extern "C" int lecqmc_ctx_destroy(lecqmc_ctx *c) {
  if (!c) return 0;
  if (c->live_walkers > 0) return fail(LECQMC_ESTATE, "context still owns %d walker(s)", c->live_walkers);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->d_batch) (void)hipFree(c->d_batch);
  for (WalkerDesc *d : c->old_batches) (void)hipFree(d);
  for (auto &r : c->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return 0;
}

extern "C" int lecqmc_ctx_synchronize(lecqmc_ctx *c) {
  if (!c) return fail(LECQMC_EINVAL, "null context");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  return 0;
}

extern "C" int lecqmc_ctx_query(lecqmc_ctx *c) {
  if (!c) return fail(LECQMC_EINVAL, "null context");
  HIPCHK(hipSetDevice(c->device));
  const hipError_t e = hipStreamQuery(c->stream);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();   // not an error: work is still in flight
    return 0;
  }
  return fail(LECQMC_EDEVICE, "hipStreamQuery: %s", hipGetErrorString(e));
}

extern "C" size_t lecqmc_ctx_bytes_in_use(const lecqmc_ctx *c) { return c ? c->used : 0; }

extern "C" int lecqmc_ctx_set_timing(lecqmc_ctx *c, int32_t enable) {
  if (!c) return fail(LECQMC_EINVAL, "null context");
  c->timing = enable != 0;
  return 0;
}

extern "C" int lecqmc_ctx_phase_times(lecqmc_ctx *c, double ms[3], int64_t counts[3]) {
  if (!c || !ms || !counts) return fail(LECQMC_EINVAL, "null argument");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int p = 0; p < 3; ++p) { ms[p] = 0.0; counts[p] = 0; }
  for (auto &r : c->recs) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.phase] += t;
    counts[r.phase] += 1;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return 0;
}

// ---------------------------------------------------------------------------
// walker
// ---------------------------------------------------------------------------
// Status of the walker's last kernels: a singular inverse or QR breakdown
// (bit 2, kept: the chain's numbers are no longer trusted) or a wrap error
// above wrap_tol on a measuring sweep (bit 3, cleared once reported: the
// walker stays valid and the caller may lower n_stab).  sc_out (if set)
// receives the scalars read.
static int check_status(lecqmc_walker *w, Scalars *sc_out = nullptr) {
  Scalars sc;
  HIPCHK(xfer(w->ctx, &sc, w->h.sc, sizeof sc, hipMemcpyDeviceToHost));
  if (sc_out) *sc_out = sc;
  if (sc.status & 4) return fail(LECQMC_EUNSTABLE, "singular P^T B P or QR breakdown");
  if (sc.status & 8) {
    const int st = sc.status & ~8;
    HIPCHK(xfer(w->ctx, &w->h.sc->status, &st, sizeof st, hipMemcpyHostToDevice));
    return fail(LECQMC_EUNSTABLE, "wrap error %.3e of the last measuring sweep above wrap_tol %.3e",
                sc.wrap_sweep, w->h.wrap_tol);
  }
  return 0;
}

extern "C" int lecqmc_create_walker(lecqmc_ctx *ctx, const lecqmc_lattice *lat, const lecqmc_params *par,
                                    const int8_t *fields, const int32_t *occ_up, const int32_t *occ_dn,
                                    lecqmc_walker **out) {
  if (!ctx || !out) return fail(LECQMC_EINVAL, "null context or out");
  int L = 0;
  if (int rc = validate(lat, par, &L)) return rc;
  const int N = lat->n_sites;
  const int ns = (lat->sublattice && lat->n_sublattices > 0) ? lat->n_sublattices : 1;
  const int ne[2] = {par->n_up, par->n_dn};
  for (int s = 0; s < 2; ++s) {
    const int32_t *g = s == 0 ? occ_up : occ_dn;
    if (!g) continue;
    std::vector<char> used(N, 0);
    for (int a = 0; a < ne[s]; ++a) {
      if (g[a] < 0 || g[a] >= N || used[g[a]]) return fail(LECQMC_EINVAL, "bad occupation list (spin %d)", s);
      used[g[a]] = 1;
    }
  }
  const Plan p = make_plan(N, L, par->n_stab, ne[0], ne[1], lat->n_bonds, lat->n_colors, ns,
                           par->precision == LECQMC_MIXED);
  if (ctx->budget && ctx->used + p.total > ctx->budget)
    return fail(LECQMC_ENOMEM, "walker needs %zu bytes, %zu of %zu in use", p.total, ctx->used, ctx->budget);
  HIPCHK(hipSetDevice(ctx->device));
  void *dmem = nullptr;
  HIPCHK(hipMalloc(&dmem, p.total));
  char *base = (char *)dmem;

  lecqmc_walker *w = new lecqmc_walker();
  w->ctx = ctx;
  w->dmem = dmem;
  w->bytes = p.total;
  w->N = N;
  w->L = L;
  w->nblk = (L + par->n_stab - 1) / par->n_stab;
  w->ne[0] = ne[0];
  w->ne[1] = ne[1];
  w->mmax = std::max(1, std::max(ne[0], ne[1]));
  w->nobs = obs_count(N, ns);

  WalkerDesc &d = w->h;
  memset(&d, 0, sizeof d);
  d.N = N; d.L = L; d.nstab = par->n_stab; d.nblk = w->nblk; d.ncol = lat->n_colors; d.nbonds = lat->n_bonds;
  d.nsub = ns; d.ncells = lat->n_cells > 0 ? lat->n_cells : N; d.flags = par->flags; d.nobs = w->nobs;
  d.mixed = par->precision == LECQMC_MIXED ? 1 : 0;
  d.ne[0] = ne[0]; d.ne[1] = ne[1]; d.mmax = w->mmax;
  {
    int tile, chunk;
    shape_default(ne[0], ne[1], &tile, &chunk);
    auto it = ctx->tuned.find(std::make_tuple(N, ne[0], ne[1], d.mixed));
    if (it != ctx->tuned.end() && shape_valid(ne[0], ne[1], it->second.first, it->second.second)) {
      tile = it->second.first;
      chunk = it->second.second;
    }
    shape_apply(d, tile, chunk);
  }
  d.seed = par->seed; d.wid = par->walker_id;
  // Ising decoupling in the spin channel: cosh(lambda) = exp(dtau U / 2)
  const double lambda = acosh(exp(par->dtau * par->U / 2.0));
  d.elam = exp(lambda);
  d.emlam = exp(-lambda);
  d.delta_dn_s = exp(-2.0 * lambda) - 1.0;   // sigma * s = +1 flipped to -1
  d.delta_up_s = exp(2.0 * lambda) - 1.0;    // sigma * s = -1 flipped to +1
  // default tolerance of the wrap check: FP64 rounding, or FP32 propagation
  d.wrap_tol = par->wrap_tol > 0 ? par->wrap_tol : (d.mixed ? 1e-4 : 1e-8);
  d.sc = (Scalars *)(base + p.off_sc);
  d.s = (int8_t *)(base + p.off_s);
  for (int s = 0; s < 2; ++s) {
    d.occ[s] = (int *)(base + p.off_occ[s]);
    d.LS[s] = (double *)(base + p.off_LS[s]);
    d.LX[s] = (double *)(base + p.off_LX[s]);
    d.RQ[s] = (double *)(base + p.off_RQ[s]);
    d.RV[s] = (double *)(base + p.off_RV[s]);
    d.Minv[s] = (double *)(base + p.off_Minv[s]);
    d.PhiR[s] = (double *)(base + p.off_PhiR[s]);
    d.X[s] = (double *)(base + p.off_X[s]);
    d.T[s] = (double *)(base + p.off_T[s]);
    d.Aw[s] = (double *)(base + p.off_Aw[s]);
  }
  d.mpart = (double *)(base + p.off_mpart);
  d.mscr = (double *)(base + p.off_mscr);
  d.mscr_stride = p.mscr_stride;
  d.fq = (double *)(base + p.off_fq);
  d.fw = (double *)(base + p.off_fw);
  d.fVp = (double *)(base + p.off_fVp);
  d.fgc = (double *)(base + p.off_fgc);
  d.fgs = (double *)(base + p.off_fgs);
  d.fv = (double *)(base + p.off_fv);
  d.frho = (double *)(base + p.off_frho);
  d.fmark = (int *)(base + p.off_fmark);
  d.obs = (double *)(base + p.off_obs);
  d.dbg = (double *)(base + p.off_dbg);
  d.bigm = (double *)(base + p.off_bigm);
  d.dch = (double *)(base + p.off_dch);
  int *col_start = (int *)(base + p.off_col);
  int *bi = (int *)(base + p.off_bi);
  int *bj = (int *)(base + p.off_bj);
  double *bdiag = (double *)(base + p.off_bdiag);
  double *boff = (double *)(base + p.off_boff);
  double *bh = (double *)(base + p.off_bh);
  double *epsf = (double *)(base + p.off_epsf);
  double *eps = (double *)(base + p.off_eps);
  int *sub = (int *)(base + p.off_sub);
  d.col_start = col_start; d.bi = bi; d.bj = bj; d.bdiag = bdiag; d.boff = boff; d.bh = bh;
  d.eps_fac = epsf; d.eps = eps; d.sub = sub;
  w->d_desc = (WalkerDesc *)(base + p.off_desc);

  // model tables: bonds grouped by colour (input order inside a colour),
  // 2x2 bond exponential e^{-dtau h sigma_x} = cosh(dtau h) 1 - sinh(dtau h) sigma_x
  std::vector<int> hcol(lat->n_colors + 1), hbi, hbj;
  std::vector<double> hdiag, hoff, hh;
  for (int c = 0; c < lat->n_colors; ++c) {
    hcol[c] = (int)hbi.size();
    for (int b = 0; b < lat->n_bonds; ++b) {
      if (lat->bond_color[b] != c) continue;
      const double h = lat->bond_h[b];
      hbi.push_back(lat->bond_i[b]);
      hbj.push_back(lat->bond_j[b]);
      hdiag.push_back(cosh(par->dtau * h));
      hoff.push_back(-sinh(par->dtau * h));
      hh.push_back(h);
    }
  }
  hcol[lat->n_colors] = (int)hbi.size();
  // compact copy: packed site pair and an index into the distinct coefficients
  std::vector<int> hbij(hbi.size());
  std::vector<uint8_t> hbci(hbi.size());
  std::vector<double> hcoef;
  int ncoef = N <= 65535 ? 0 : -1;
  for (size_t b = 0; b < hbi.size() && ncoef >= 0; ++b) {
    hbij[b] = hbi[b] | (hbj[b] << 16);
    int ci = -1;
    for (int q = 0; q < ncoef; ++q)
      if (hcoef[2 * q] == hdiag[b] && hcoef[2 * q + 1] == hoff[b]) { ci = q; break; }
    if (ci < 0) {
      if (ncoef == kMaxCoef) { ncoef = -1; break; }
      hcoef.push_back(hdiag[b]);
      hcoef.push_back(hoff[b]);
      ci = ncoef++;
    }
    hbci[b] = (uint8_t)ci;
  }
  d.ncoef = ncoef > 0 ? ncoef : 0;
  d.bond_words = d.ncoef > 0 ? 2 * 2 * kMaxCoef + (int)hbi.size() + ((int)hbi.size() + 3) / 4 : 0;
  d.bij = (const int *)(base + p.off_bij);
  d.bci = (const uint8_t *)(base + p.off_bci);
  d.coef = (const double *)(base + p.off_coef);
  std::vector<double> hepsf(N), heps(N);
  std::vector<int> hsub(N);
  for (int i = 0; i < N; ++i) {
    heps[i] = lat->onsite ? lat->onsite[i] : 0.0;
    hepsf[i] = exp(-par->dtau * heps[i]);
    hsub[i] = lat->sublattice ? lat->sublattice[i] : 0;
  }
  auto cleanup = [&](int rc) { (void)hipFree(dmem); delete w; return rc; };
  auto up = [&](void *dst, const void *src, size_t n) -> hipError_t {
    return n ? xfer(ctx, dst, src, n, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e = zero(ctx, dmem, p.total);
  if (e == hipSuccess) e = up(col_start, hcol.data(), sizeof(int) * hcol.size());
  if (e == hipSuccess) e = up(bi, hbi.data(), sizeof(int) * hbi.size());
  if (e == hipSuccess) e = up(bj, hbj.data(), sizeof(int) * hbj.size());
  if (e == hipSuccess) e = up(bdiag, hdiag.data(), sizeof(double) * hdiag.size());
  if (e == hipSuccess) e = up(boff, hoff.data(), sizeof(double) * hoff.size());
  if (e == hipSuccess) e = up(bh, hh.data(), sizeof(double) * hh.size());
  if (e == hipSuccess) e = up(epsf, hepsf.data(), sizeof(double) * N);
  if (e == hipSuccess) e = up(eps, heps.data(), sizeof(double) * N);
  if (e == hipSuccess) e = up(sub, hsub.data(), sizeof(int) * N);
  if (e == hipSuccess && d.ncoef > 0) e = up((void *)d.bij, hbij.data(), sizeof(int) * hbij.size());
  if (e == hipSuccess && d.ncoef > 0) e = up((void *)d.bci, hbci.data(), hbci.size());
  if (e == hipSuccess && d.ncoef > 0) e = up((void *)d.coef, hcoef.data(), sizeof(double) * hcoef.size());
  if (e == hipSuccess && fields) {
    std::vector<int8_t> f((size_t)L * N);
    for (size_t t = 0; t < f.size(); ++t) f[t] = fields[t] > 0 ? 1 : -1;
    e = up(d.s, f.data(), f.size());
  }
  if (e == hipSuccess && occ_up) e = up(d.occ[0], occ_up, sizeof(int) * ne[0]);
  if (e == hipSuccess && occ_dn) e = up(d.occ[1], occ_dn, sizeof(int) * ne[1]);
  if (e == hipSuccess) e = up(w->d_desc, &d, sizeof d);
  if (e != hipSuccess) return cleanup(fail(LECQMC_EDEVICE, "upload: %s", hipGetErrorString(e)));
  const int draw_occ = (occ_up ? 0 : 1) | (occ_dn ? 0 : 2);
  if (!fields || draw_occ) e = launch_init(w->d_desc, fields ? 0 : 1, draw_occ, ctx->stream);
  const LaunchCfg cf = launch_cfg(&w, 1);
  if (e == hipSuccess) e = launch_fresh_weight(w->d_desc, 1, cf.fresh, 1, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return cleanup(fail(LECQMC_EDEVICE, "init: %s", hipGetErrorString(e)));
  ctx->used += p.total;
  ctx->live_walkers += 1;
  if (int rc = check_status(w)) { lecqmc_destroy_walker(w); return rc; }
  *out = w;
  return 0;
}

extern "C" int lecqmc_destroy_walker(lecqmc_walker *w) {
  if (!w) return 0;
  if (w->batches > 0) return fail(LECQMC_ESTATE, "walker still belongs to %d batch(es)", w->batches);
  (void)hipSetDevice(w->ctx->device);
  (void)hipStreamSynchronize(w->ctx->stream);
  (void)hipFree(w->dmem);
  w->ctx->used -= w->bytes;
  w->ctx->live_walkers -= 1;
  delete w;
  return 0;
}

extern "C" int lecqmc_sweep(lecqmc_walker *w, int32_t n_sweeps, int32_t do_measure) {
  if (!w || n_sweeps < 0) return fail(LECQMC_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(w->ctx->device));
  hipStream_t st = w->ctx->stream;
  lecqmc_ctx *c = w->ctx;
  const LaunchCfg cf = launch_cfg(&w, 1);
  for (int t = 0; t < n_sweeps; ++t) {
    HIPCHK(timed(c, 0, [&] { return launch_left_stack(w->d_desc, 1, cf.left, cf.mixed, st); }));
    HIPCHK(timed(c, 1, [&] { return launch_forward(w->d_desc, 1, cf.fwd, cf.tile, do_measure, cf.mixed, st); }));
    if (do_measure) HIPCHK(launch_measure(w->d_desc, 1, cf.slots, cf.meas, st));
    HIPCHK(timed(c, 2, [&] { return launch_fock(w->d_desc, 1, cf.fock, cf.mixed, st); }));
  }
  return 0;
}

// Walkers of a batch call in launch order (FP64 first, then mixed precision),
// after the checks both batch entry points share.
static int batch_order(lecqmc_walker *const *ws, int32_t n, int32_t n_sweeps, std::vector<lecqmc_walker *> &order,
                       int *n64) {
  if (!ws || n <= 0 || n_sweeps < 0 || !ws[0]) return fail(LECQMC_EINVAL, "bad arguments");
  lecqmc_ctx *c = ws[0]->ctx;
  order.clear();
  for (int pass = 0; pass < 2; ++pass)
    for (int t = 0; t < n; ++t) {
      if (!ws[t] || ws[t]->ctx != c) return fail(LECQMC_EINVAL, "walkers of a batch must share one context");
      if (ws[t]->h.mixed == pass) order.push_back(ws[t]);
    }
  {
    // two workgroups of every phase would update one walker's state at once
    std::vector<lecqmc_walker *> sorted(order);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(LECQMC_EINVAL, "a walker appears twice in the batch");
  }
  *n64 = 0;
  for (lecqmc_walker *w : order) *n64 += w->h.mixed ? 0 : 1;
  return 0;
}

// Upload the descriptors of `order` to d (device) and run the sweeps, one
// launch per precision group and phase.  timing: record phase events.
static int batch_run(lecqmc_ctx *c, const std::vector<lecqmc_walker *> &order, int n64, WalkerDesc *d,
                     int32_t n_sweeps, int32_t do_measure, bool timing) {
  const int n = (int)order.size();
  std::vector<WalkerDesc> hd(n);
  for (int t = 0; t < n; ++t) hd[t] = order[t]->h;
  struct Group {
    const WalkerDesc *d;
    int n;
    LaunchCfg cf;
  };
  std::vector<Group> groups;
  if (n64 > 0) groups.push_back({d, n64, launch_cfg(order.data(), n64)});
  if (n > n64) groups.push_back({d + n64, n - n64, launch_cfg(order.data() + n64, n - n64)});
  for (const Group &g : groups)
    if (!g.cf.fits) return fail(LECQMC_EINVAL, "the chain staging of these walkers does not fit one launch's LDS; "
                                               "sweep them in separate batches or give them smaller chunks");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(xfer(c, d, hd.data(), sizeof(WalkerDesc) * n, hipMemcpyHostToDevice));
  auto each = [&](auto &&launch) {
    for (const Group &g : groups) {
      const hipError_t e = launch(g);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto phase = [&](int ph, auto &&launch) { return timing ? timed(c, ph, launch) : launch(); };
  for (int t = 0; t < n_sweeps; ++t) {
    HIPCHK(phase(0, [&] { return each([&](const Group &g) {
      return launch_left_stack(g.d, g.n, g.cf.left, g.cf.mixed, c->stream); }); }));
    HIPCHK(phase(1, [&] { return each([&](const Group &g) {
      return launch_forward(g.d, g.n, g.cf.fwd, g.cf.tile, do_measure, g.cf.mixed, c->stream); }); }));
    if (do_measure)
      HIPCHK(each([&](const Group &g) { return launch_measure(g.d, g.n, g.cf.slots, g.cf.meas, c->stream); }));
    HIPCHK(phase(2, [&] { return each([&](const Group &g) {
      return launch_fock(g.d, g.n, g.cf.fock, g.cf.mixed, c->stream); }); }));
  }
  return 0;
}

extern "C" int lecqmc_sweep_batch(lecqmc_walker *const *ws, int32_t n, int32_t n_sweeps, int32_t do_measure) {
  std::vector<lecqmc_walker *> order;
  int n64 = 0;
  if (int rc = batch_order(ws, n, n_sweeps, order, &n64)) return rc;
  lecqmc_ctx *c = order[0]->ctx;
  HIPCHK(hipSetDevice(c->device));
  if (c->batch_cap < n) {
    const int cap = std::max(n, std::max(64, 2 * c->batch_cap));
    WalkerDesc *nd = nullptr;
    HIPCHK(hipMalloc(&nd, sizeof(WalkerDesc) * cap));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->d_batch) c->old_batches.push_back(c->d_batch);
    c->d_batch = nd;
    c->batch_cap = cap;
  }
  return batch_run(c, order, n64, c->d_batch, n_sweeps, do_measure, true);
}

// The same sweeps with the descriptors staged in the device's static array
// (no allocation of any kind; phase timing is not recorded).
extern "C" int lecqmc_sweep_batch_static(lecqmc_walker *const *ws, int32_t n, int32_t n_sweeps,
                                         int32_t do_measure) {
  if (n > kStaticMaxWalkers)
    return fail(LECQMC_EINVAL, "sweep_batch_static: %d walkers, at most %d", n, kStaticMaxWalkers);
  std::vector<lecqmc_walker *> order;
  order.reserve(n > 0 ? n : 0);
  int n64 = 0;
  if (int rc = batch_order(ws, n, n_sweeps, order, &n64)) return rc;
  lecqmc_ctx *c = order[0]->ctx;
  HIPCHK(hipSetDevice(c->device));
  return batch_run(c, order, n64, c->scratch_desc, n_sweeps, do_measure, false);
}

// ---------------------------------------------------------------------------
// fixed batches: descriptors uploaded once, sweeps that only launch kernels
// ---------------------------------------------------------------------------
struct lecqmc_batch {
  lecqmc_ctx *ctx;
  std::vector<lecqmc_walker *> ws;
  WalkerDesc *d;
  int n, n64;
  LaunchCfg cf64, cfmx;
};

extern "C" int lecqmc_batch_create(lecqmc_walker *const *ws, int32_t n, lecqmc_batch **out) {
  if (!ws || n <= 0 || !out) return fail(LECQMC_EINVAL, "bad arguments");
  lecqmc_ctx *c = ws[0] ? ws[0]->ctx : nullptr;
  std::vector<lecqmc_walker *> order;
  for (int pass = 0; pass < 2; ++pass)
    for (int t = 0; t < n; ++t) {
      if (!ws[t] || ws[t]->ctx != c) return fail(LECQMC_EINVAL, "walkers of a batch must share one context");
      if (ws[t]->h.mixed == pass) order.push_back(ws[t]);
    }
  for (int t = 0; t < n; ++t)
    for (int u = t + 1; u < n; ++u)
      if (order[t] == order[u]) return fail(LECQMC_EINVAL, "a walker appears twice in the batch");
  HIPCHK(hipSetDevice(c->device));
  std::vector<WalkerDesc> hd(n);
  int n64 = 0;
  for (int t = 0; t < n; ++t) {
    hd[t] = order[t]->h;
    n64 += order[t]->h.mixed ? 0 : 1;
  }
  WalkerDesc *d = nullptr;
  HIPCHK(hipMalloc(&d, sizeof(WalkerDesc) * n));
  const hipError_t e = xfer(c, d, hd.data(), sizeof(WalkerDesc) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(LECQMC_EDEVICE, "upload: %s", hipGetErrorString(e));
  }
  lecqmc_batch *b = new lecqmc_batch();
  b->ctx = c;
  b->ws = order;
  b->d = d;
  b->n = n;
  b->n64 = n64;
  if (n64 > 0) b->cf64 = launch_cfg(order.data(), n64);
  if (n > n64) b->cfmx = launch_cfg(order.data() + n64, n - n64);
  if ((n64 > 0 && !b->cf64.fits) || (n > n64 && !b->cfmx.fits)) {
    (void)hipFree(d);
    delete b;
    return fail(LECQMC_EINVAL, "the chain staging of these walkers does not fit one launch's LDS; "
                               "batch them separately or give them smaller chunks");
  }
  for (lecqmc_walker *w : order) w->batches += 1;
  *out = b;
  return 0;
}

extern "C" int lecqmc_batch_sweep(lecqmc_batch *b, int32_t n_sweeps, int32_t do_measure) {
  if (!b || n_sweeps < 0) return fail(LECQMC_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(b->ctx->device));
  hipStream_t st = b->ctx->stream;
  for (int t = 0; t < n_sweeps; ++t)
    for (int g = 0; g < 2; ++g) {
      const int gn = g == 0 ? b->n64 : b->n - b->n64;
      if (gn == 0) continue;
      const WalkerDesc *d = g == 0 ? b->d : b->d + b->n64;
      const LaunchCfg &cf = g == 0 ? b->cf64 : b->cfmx;
      HIPCHK(launch_left_stack(d, gn, cf.left, cf.mixed, st));
      HIPCHK(launch_forward(d, gn, cf.fwd, cf.tile, do_measure, cf.mixed, st));
      if (do_measure) HIPCHK(launch_measure(d, gn, cf.slots, cf.meas, st));
      HIPCHK(launch_fock(d, gn, cf.fock, cf.mixed, st));
    }
  return 0;
}

extern "C" int lecqmc_batch_destroy(lecqmc_batch *b) {
  if (!b) return 0;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  (void)hipFree(b->d);
  for (lecqmc_walker *w : b->ws) w->batches -= 1;
  delete b;
  return 0;
}

// ---------------------------------------------------------------------------
// flip-chain shapes and the autotuner
// ---------------------------------------------------------------------------
extern "C" int lecqmc_get_shape(const lecqmc_walker *w, int32_t *tile, int32_t *chunk) {
  if (!w || !tile || !chunk) return fail(LECQMC_EINVAL, "null argument");
  *tile = w->h.tile;
  *chunk = w->h.chunk;
  return 0;
}

static int set_shape(lecqmc_walker *w, int tile, int chunk) {
  shape_apply(w->h, tile, chunk);
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(xfer(w->ctx, w->d_desc, &w->h, sizeof(WalkerDesc), hipMemcpyHostToDevice));
  return 0;
}

extern "C" int lecqmc_set_shape(lecqmc_walker *w, int32_t tile, int32_t chunk) {
  if (!w) return fail(LECQMC_EINVAL, "null walker");
  if (!shape_valid(w->ne[0], w->ne[1], tile, chunk))
    return fail(LECQMC_EINVAL, "shape (tile %d, chunk %d) not valid for Ne = %d", tile, chunk, w->mmax);
  if (w->batches > 0) return fail(LECQMC_ESTATE, "walker belongs to %d batch(es)", w->batches);
  HIPCHK(hipSetDevice(w->ctx->device));
  return set_shape(w, tile, chunk);
}

// Every candidate shape runs one whole forward pass of every walker it is
// valid for, from the same saved state (fields and scalars: the rest of a
// walker's device state is rebuilt by the next sweep), timed per walker by
// the kernel's own wall clock.  The state is restored afterwards, so tuning
// leaves the Markov chains where they were.
constexpr int kTiles = 6;
extern "C" int lecqmc_autotune(lecqmc_walker *const *ws, int32_t n, int32_t *tile_out, int32_t *chunk_out,
                               double *fwd_ms_out) {
  if (!ws || n <= 0) return fail(LECQMC_EINVAL, "bad arguments");
  lecqmc_ctx *c = ws[0] ? ws[0]->ctx : nullptr;
  for (int t = 0; t < n; ++t) {
    if (!ws[t] || ws[t]->ctx != c) return fail(LECQMC_EINVAL, "walkers must share one context");
    if (ws[t]->batches > 0) return fail(LECQMC_ESTATE, "walker %d belongs to a batch", t);
    for (int u = 0; u < t; ++u)
      if (ws[u] == ws[t]) return fail(LECQMC_EINVAL, "a walker appears twice");
  }
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  int rate_khz = 0;
  HIPCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
  if (rate_khz <= 0) return fail(LECQMC_EDEVICE, "no wall-clock rate");
  // saved state: fields and scalars of every walker
  std::vector<size_t> off(n + 1, 0);
  for (int t = 0; t < n; ++t)
    off[t + 1] = off[t] + align256((size_t)ws[t]->L * ws[t]->N) + align256(sizeof(Scalars));
  char *snap = nullptr;
  HIPCHK(hipMalloc(&snap, off[n]));
  std::vector<WalkerDesc> hd;
  WalkerDesc *dd = nullptr;
  hipError_t e = hipMalloc(&dd, sizeof(WalkerDesc) * n);
  std::vector<int> cur_tile(n), cur_chunk(n);
  // per shape key and candidate: summed milliseconds of its walkers (< 0: not run)
  using Key = std::tuple<int, int, int, int>;
  auto key_of = [](const lecqmc_walker *w) { return std::make_tuple(w->N, w->ne[0], w->ne[1], w->h.mixed); };
  std::map<Key, std::vector<double>> tot;
  std::vector<std::vector<double>> wms(n, std::vector<double>(4 * kTiles, -1.0));
  for (int t = 0; t < n; ++t) tot[key_of(ws[t])].assign(4 * kTiles, -1.0);
  auto restore = [&](int t) {
    const size_t nf = (size_t)ws[t]->L * ws[t]->N;
    hipError_t r = hipMemcpyAsync(ws[t]->h.s, snap + off[t], nf, hipMemcpyDeviceToDevice, st);
    if (r == hipSuccess)
      r = hipMemcpyAsync(ws[t]->h.sc, snap + off[t] + align256(nf), sizeof(Scalars), hipMemcpyDeviceToDevice, st);
    return r;
  };
  for (int t = 0; t < n; ++t) {
    cur_tile[t] = ws[t]->h.tile;
    cur_chunk[t] = ws[t]->h.chunk;
  }
  // the left states of the current fields (they do not depend on the shape)
  for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
    std::vector<lecqmc_walker *> g;
    for (int t = 0; t < n; ++t)
      if (ws[t]->h.mixed == pass) g.push_back(ws[t]);
    if (g.empty()) continue;
    hd.clear();
    for (auto *w : g) hd.push_back(w->h);
    e = xfer(c, dd, hd.data(), sizeof(WalkerDesc) * hd.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_left_stack(dd, (int)g.size(), launch_cfg(g.data(), (int)g.size()).left, pass, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  for (int t = 0; t < n && e == hipSuccess; ++t) {
    const size_t nf = (size_t)ws[t]->L * ws[t]->N;
    e = hipMemcpyAsync(snap + off[t], ws[t]->h.s, nf, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(snap + off[t] + align256(nf), ws[t]->h.sc, sizeof(Scalars), hipMemcpyDeviceToDevice, st);
  }
  static const int tiles[kTiles] = {1, 2, 4, 0, kDelayed, kMfma}, chunks[4] = {4, 8, 16, 32};
  for (int ti = 0; ti < kTiles && e == hipSuccess; ++ti)
    for (int ci = 0; ci < 4 && e == hipSuccess; ++ci)
      for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        std::vector<lecqmc_walker *> g;
        std::vector<int> idx;
        for (int t = 0; t < n; ++t)
          if (ws[t]->h.mixed == pass && shape_valid(ws[t]->ne[0], ws[t]->ne[1], tiles[ti], chunks[ci])) {
            g.push_back(ws[t]);
            idx.push_back(t);
          }
        if (g.empty()) continue;
        hd.clear();
        for (auto *w : g) {
          shape_apply(w->h, tiles[ti], chunks[ci]);
          hd.push_back(w->h);
        }
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = xfer(c, dd, hd.data(), sizeof(WalkerDesc) * hd.size(), hipMemcpyHostToDevice);
        const LaunchCfg cf = launch_cfg(g.data(), (int)g.size());
        if (!cf.fits) continue;   // this candidate cannot run these walkers in one launch
        if (e == hipSuccess) e = launch_forward(dd, (int)g.size(), cf.fwd, cf.tile, 0, pass, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        for (size_t q = 0; q < g.size() && e == hipSuccess; ++q) {
          long long ticks = 0;
          e = xfer(c, &ticks, &g[q]->h.sc->fwd_ticks, sizeof ticks, hipMemcpyDeviceToHost);
          const double ms = (double)ticks / (double)rate_khz;
          const int t = idx[q], cand = ti * 4 + ci;
          if (e == hipSuccess) {
            wms[t][cand] = ms;
            double &sum = tot[key_of(ws[t])][cand];
            sum = (sum < 0.0 ? 0.0 : sum) + ms;
            e = restore(t);
          }
        }
      }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dd);
  (void)hipFree(snap);
  // one shape per key: the candidate with the least summed time over the
  // key's walkers (the current shapes if tuning failed)
  const bool ok = e == hipSuccess;
  std::map<Key, int> best;
  for (auto &kv : tot) {
    int bc = -1;
    for (int q = 0; q < 4 * kTiles; ++q)
      if (kv.second[q] >= 0.0 && (bc < 0 || kv.second[q] < kv.second[bc])) bc = q;
    best[kv.first] = bc;
  }
  for (int t = 0; t < n; ++t) {
    const int bc = ok ? best[key_of(ws[t])] : -1;
    const int tile = bc >= 0 ? tiles[bc / 4] : cur_tile[t], chunk = bc >= 0 ? chunks[bc % 4] : cur_chunk[t];
    if (int rc = set_shape(ws[t], tile, chunk)) return rc;
    if (bc >= 0) c->tuned[key_of(ws[t])] = {tile, chunk};
    if (tile_out) tile_out[t] = tile;
    if (chunk_out) chunk_out[t] = chunk;
    if (fwd_ms_out) fwd_ms_out[t] = bc >= 0 ? wms[t][bc] : -1.0;
  }
  if (e != hipSuccess) return fail(LECQMC_EDEVICE, "autotune: %s", hipGetErrorString(e));
  return 0;
}

extern "C" int lecqmc_log_weight(lecqmc_walker *w, double *log_abs_w, int32_t *sign) {
  if (!w || !log_abs_w || !sign) return fail(LECQMC_EINVAL, "null argument");
  HIPCHK(hipSetDevice(w->ctx->device));
  const LaunchCfg cf = launch_cfg(&w, 1);
  HIPCHK(launch_fresh_weight(w->d_desc, 1, cf.fresh, 0, w->ctx->stream));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  Scalars sc;
  const int rc = check_status(w, &sc);
  *log_abs_w = sc.fresh_logw;
  *sign = sc.fresh_sign;
  return rc;
}

extern "C" int lecqmc_tracked_weight(lecqmc_walker *w, double *log_abs_w, int32_t *sign) {
  if (!w || !log_abs_w || !sign) return fail(LECQMC_EINVAL, "null argument");
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  Scalars sc;
  const int rc = check_status(w, &sc);
  *log_abs_w = sc.logw + sc.fock_logw[0] + sc.fock_logw[1];
  *sign = sc.sign * sc.fock_sign[0] * sc.fock_sign[1];
  return rc;
}

extern "C" int64_t lecqmc_obs_size(const lecqmc_walker *w) { return w ? w->nobs : 0; }

extern "C" int lecqmc_measure(lecqmc_walker *w, double *out, int64_t n) {
  if (!w || !out || n < w->nobs) return fail(LECQMC_EINVAL, "output too small (%d needed)", w ? w->nobs : 0);
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(xfer(w->ctx, out, w->h.obs, sizeof(double) * w->nobs, hipMemcpyDeviceToHost));
  return check_status(w);
}

extern "C" int lecqmc_reset_measure(lecqmc_walker *w) {
  if (!w) return fail(LECQMC_EINVAL, "null walker");
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(zero(w->ctx, w->h.obs, sizeof(double) * w->nobs));
  return 0;
}

extern "C" int lecqmc_get_stats(lecqmc_walker *w, lecqmc_sweep_stats *st) {
  if (!w || !st) return fail(LECQMC_EINVAL, "null argument");
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  Scalars sc;
  const int rc = check_status(w, &sc);
  if (rc == LECQMC_EDEVICE) return rc;
  st->flip_attempts = sc.flip_att;
  st->flip_accepts = sc.flip_acc;
  st->swap_attempts = sc.swap_att[0] + sc.swap_att[1];
  st->swap_accepts = sc.swap_acc[0] + sc.swap_acc[1];
  st->max_wrap_err = sc.max_wrap;
  st->logw_drift = sc.logw_drift;
  st->qr_shifted = sc.qr_shifted;
  st->sweeps = sc.sweep;
  st->near_ties = sc.near_ties + sc.swap_near[0] + sc.swap_near[1];
  return rc;
}

extern "C" int lecqmc_get_state(lecqmc_walker *w, int8_t *fields, int32_t *occ_up, int32_t *occ_dn,
                                uint64_t *sweep_counter) {
  if (!w) return fail(LECQMC_EINVAL, "null walker");
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  if (fields) HIPCHK(xfer(w->ctx, fields, w->h.s, (size_t)w->L * w->N, hipMemcpyDeviceToHost));
  if (occ_up && w->ne[0]) HIPCHK(xfer(w->ctx, occ_up, w->h.occ[0], sizeof(int) * w->ne[0], hipMemcpyDeviceToHost));
  if (occ_dn && w->ne[1]) HIPCHK(xfer(w->ctx, occ_dn, w->h.occ[1], sizeof(int) * w->ne[1], hipMemcpyDeviceToHost));
  if (sweep_counter) {
    Scalars sc;
    HIPCHK(xfer(w->ctx, &sc, w->h.sc, sizeof sc, hipMemcpyDeviceToHost));
    *sweep_counter = sc.sweep;
  }
  return 0;
}

extern "C" int lecqmc_set_state(lecqmc_walker *w, const int8_t *fields, const int32_t *occ_up,
                                const int32_t *occ_dn, uint64_t sweep_counter) {
  if (!w) return fail(LECQMC_EINVAL, "null walker");
  for (int s = 0; s < 2; ++s) {
    const int32_t *g = s == 0 ? occ_up : occ_dn;
    if (!g) continue;
    std::vector<char> used(w->N, 0);
    for (int a = 0; a < w->ne[s]; ++a) {
      if (g[a] < 0 || g[a] >= w->N || used[g[a]]) return fail(LECQMC_EINVAL, "bad occupation list");
      used[g[a]] = 1;
    }
  }
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  if (fields) {
    std::vector<int8_t> f((size_t)w->L * w->N);
    for (size_t t = 0; t < f.size(); ++t) f[t] = fields[t] > 0 ? 1 : -1;
    HIPCHK(xfer(w->ctx, w->h.s, f.data(), f.size(), hipMemcpyHostToDevice));
  }
  if (occ_up && w->ne[0]) HIPCHK(xfer(w->ctx, w->h.occ[0], occ_up, sizeof(int) * w->ne[0], hipMemcpyHostToDevice));
  if (occ_dn && w->ne[1]) HIPCHK(xfer(w->ctx, w->h.occ[1], occ_dn, sizeof(int) * w->ne[1], hipMemcpyHostToDevice));
  Scalars sc;
  HIPCHK(xfer(w->ctx, &sc, w->h.sc, sizeof sc, hipMemcpyDeviceToHost));
  sc.sweep = sweep_counter;
  HIPCHK(xfer(w->ctx, w->h.sc, &sc, sizeof sc, hipMemcpyHostToDevice));
  const LaunchCfg cf = launch_cfg(&w, 1);
  HIPCHK(launch_fresh_weight(w->d_desc, 1, cf.fresh, 1, w->ctx->stream));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  return check_status(w);
}

extern "C" int lecqmc_green(lecqmc_walker *w, int32_t boundary, int32_t spin, double *G) {
  if (!w || !G || boundary < 0 || boundary > w->L || spin < 0 || spin > 1) return fail(LECQMC_EINVAL, "bad arguments");
  if (w->N > 8192) return fail(LECQMC_EINVAL, "green: N x N output limited to N <= 8192");
  // the N x N staging buffer lives for this call only and counts against
  // the context's budget while it does
  lecqmc_ctx *c = w->ctx;
  const size_t bytes = sizeof(double) * (size_t)w->N * w->N;
  if (c->budget && c->used + bytes > c->budget)
    return fail(LECQMC_ENOMEM, "green: %zu bytes of staging, %zu of %zu in use", bytes, c->used, c->budget);
  HIPCHK(hipSetDevice(c->device));
  double *dg = nullptr;
  HIPCHK(hipMalloc(&dg, bytes));
  c->used += bytes;
  hipError_t e = launch_green(w->d_desc, w->mmax, boundary, spin, dg, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = xfer(c, G, dg, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(dg);
  c->used -= bytes;
  if (e != hipSuccess) return fail(LECQMC_EDEVICE, "green: %s", hipGetErrorString(e));
  return check_status(w);
}

extern "C" int lecqmc_flip_ratio(lecqmc_walker *w, int32_t slice, int32_t site, double *ratio) {
  if (!w || !ratio || slice < 0 || slice >= w->L || site < 0 || site >= w->N) return fail(LECQMC_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(launch_flip_ratio(w->d_desc, w->mmax, slice, site, w->ctx->stream));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(xfer(w->ctx, ratio, w->h.dbg, sizeof(double), hipMemcpyDeviceToHost));
  return check_status(w);
}

extern "C" int lecqmc_swap_ratio(lecqmc_walker *w, int32_t spin, int32_t k, int32_t j, double *ratio) {
  if (!w || !ratio || spin < 0 || spin > 1) return fail(LECQMC_EINVAL, "bad arguments");
  const int ne = w->ne[spin];
  if (ne == 0 || ne == w->N || k < 0 || k >= ne || j < 0 || j >= w->N) return fail(LECQMC_EINVAL, "bad swap indices");
  std::vector<int32_t> occ(ne);
  HIPCHK(hipSetDevice(w->ctx->device));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(xfer(w->ctx, occ.data(), w->h.occ[spin], sizeof(int) * ne, hipMemcpyDeviceToHost));
  for (int a = 0; a < ne; ++a)
    if (occ[a] == j) return fail(LECQMC_EINVAL, "site %d is occupied", j);
  HIPCHK(launch_swap_ratio(w->d_desc, w->mmax, spin, k, j, w->ctx->stream));
  HIPCHK(hipStreamSynchronize(w->ctx->stream));
  HIPCHK(xfer(w->ctx, ratio, w->h.dbg, sizeof(double), hipMemcpyDeviceToHost));
  return check_status(w);
}

// ---------------------------------------------------------------------------
// Constrained-path inner walk (SM Sec. VI): a population of random walkers of
// one Fock state, guided by the U = 0 trial walker of the same state.
// ---------------------------------------------------------------------------
struct lecqmc_cp {
  lecqmc_ctx *ctx;
  lecqmc_walker *trial;   // U = 0, the Fock state eta: tables and the backward trial states
  CpDesc d;               // d.cur = the live walker states
  CpState other;          // the comb's destination
  void *dmem;
  size_t bytes;
  int N, L, nw, pc_every;
  LdsPlan plan;
};

extern "C" int lecqmc_cp_create(lecqmc_ctx *ctx, const lecqmc_lattice *lat, const lecqmc_params *par,
                                const int32_t *occ_up, const int32_t *occ_dn, int32_t n_walkers, int32_t mode,
                                int32_t pc_every, lecqmc_cp **out) {
  if (!ctx || !out || !par || !occ_up || !occ_dn) return fail(LECQMC_EINVAL, "null argument");
  if (n_walkers < 1 || (mode != LECQMC_CP_IMPORTANCE && mode != LECQMC_CP_FREE) || pc_every < 0)
    return fail(LECQMC_EINVAL, "bad walker count, mode or control interval");
  if (par->precision != LECQMC_FP64) return fail(LECQMC_EINVAL, "the constrained-path walk runs in FP64 only");
  if (par->n_up > kLdsNe || par->n_dn > kLdsNe)
    return fail(LECQMC_EINVAL, "the constrained-path walk holds its inverses in LDS: Ne <= %d per spin", kLdsNe);
  lecqmc_params p0 = *par;
  p0.U = 0.0;
  p0.flags = LECQMC_NO_FLIPS | LECQMC_NO_FOCK;
  lecqmc_walker *tw = nullptr;
  if (int rc = lecqmc_create_walker(ctx, lat, &p0, nullptr, occ_up, occ_dn, &tw)) return rc;
  const int N = tw->N, L = tw->L, ne0 = tw->ne[0], ne1 = tw->ne[1];
  const int mm = std::max(std::max(ne0, ne1), 1);
  const size_t nw = (size_t)n_walkers;
  // per walker: two state sets (phi, inverse, field path, weights), QR scratch
  const size_t phi_b = (size_t)N * (ne0 + ne1) * sizeof(double);
  const size_t inv_b = (size_t)(ne0 * ne0 + ne1 * ne1) * sizeof(double);
  const size_t per = 2 * (align256(phi_b) + align256(inv_b) + align256((size_t)L * N) + 2 * sizeof(double)) +
                     align256(phi_b) + 2 * (size_t)mm * mm * sizeof(double) + sizeof(long long) + sizeof(int);
  const size_t total = nw * per + 4096;
  if (ctx->budget && ctx->used + total > ctx->budget) {
    lecqmc_destroy_walker(tw);
    return fail(LECQMC_ENOMEM, "constrained-path population needs %zu bytes, %zu of %zu in use", total, ctx->used,
                ctx->budget);
  }
  void *dmem = nullptr;
  hipError_t e = hipMalloc(&dmem, total);
  if (e != hipSuccess) {
    lecqmc_destroy_walker(tw);
    return fail(LECQMC_EDEVICE, "hipMalloc: %s", hipGetErrorString(e));
  }
  char *b = (char *)dmem;
  auto take = [&](size_t n) { char *r = b; b += align256(n); return r; };
  lecqmc_cp *c = new lecqmc_cp();
  c->ctx = ctx;
  c->trial = tw;
  c->dmem = dmem;
  c->bytes = total;
  c->N = N;
  c->L = L;
  c->nw = n_walkers;
  c->pc_every = pc_every;
  CpState *sets[2] = {&c->d.cur, &c->other};
  for (CpState *st : sets) {
    st->phi[0] = (double *)take(nw * N * ne0 * sizeof(double));
    st->phi[1] = (double *)take(nw * N * ne1 * sizeof(double));
    st->minv[0] = (double *)take(nw * ne0 * ne0 * sizeof(double));
    st->minv[1] = (double *)take(nw * ne1 * ne1 * sizeof(double));
    st->s = (int8_t *)take(nw * L * N);
    st->logw = (double *)take(nw * sizeof(double));
    st->logq = (double *)take(nw * sizeof(double));
  }
  c->d.tmp[0] = (double *)take(nw * N * ne0 * sizeof(double));
  c->d.tmp[1] = (double *)take(nw * N * ne1 * sizeof(double));
  c->d.vacc = (double *)take(nw * 2 * mm * mm * sizeof(double));
  c->d.cuts = (long long *)take(nw * sizeof(long long));
  c->d.pick = (int *)take(nw * sizeof(int));
  c->d.log_pc = (double *)take(sizeof(double));
  c->d.nw = n_walkers;
  c->d.mode = mode;
  c->d.mm = mm;
  c->d.seed = par->seed;
  const double lam = acosh(exp(par->dtau * par->U / 2.0));
  for (int sp = 0; sp < 2; ++sp)
    for (int u = 0; u < 2; ++u) {
      const double sigma = sp == 0 ? 1.0 : -1.0, s = u == 0 ? 1.0 : -1.0;
      c->d.delta[sp][u] = exp(sigma * lam * s) - 1.0;
    }
  ctx->used += total;
  const LaunchCfg cf = launch_cfg(&tw, 1);
  c->plan = LdsPlan{mm, 0, 0, cf.left.bond_words, 0, 0, 0, 0};
  if (lds_bytes(c->plan) > kLdsLimit) c->plan.bond_words = 0;   // bonds then read from device memory
  // the backward trial states X_l at every slice: the trial walker's left stack
  e = launch_left_stack(tw->d_desc, 1, cf.left, 0, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    lecqmc_cp_destroy(c);
    return fail(LECQMC_EDEVICE, "trial left stack: %s", hipGetErrorString(e));
  }
  *out = c;
  return 0;
}

extern "C" int lecqmc_cp_run(lecqmc_cp *c, uint32_t tag, double *log_r) {
  if (!c || !log_r) return fail(LECQMC_EINVAL, "null argument");
  lecqmc_ctx *ctx = c->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  HIPCHK(launch_cp_init(c->trial->d_desc, c->d, st));
  HIPCHK(hipMemsetAsync(c->d.log_pc, 0, sizeof(double), st));
  for (int l = 1; l <= c->L;) {
    int le = c->L;
    if (c->pc_every > 0) le = std::min(c->L, ((l - 1) / c->pc_every + 1) * c->pc_every);
    HIPCHK(timed(ctx, 1, [&] { return launch_cp_walk(c->trial->d_desc, c->d, c->plan, l, le, tag, st); }));
    if (c->pc_every > 0 && le % c->pc_every == 0 && le < c->L) {
      HIPCHK(launch_cp_comb(c->d, c->other, c->trial->d_desc, le, tag, st));
      std::swap(c->d.cur, c->other);
    }
    l = le + 1;
  }
  std::vector<double> lw(c->nw);
  double lpc = 0.0;
  HIPCHK(hipMemcpyAsync(lw.data(), c->d.cur.logw, sizeof(double) * c->nw, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&lpc, c->d.log_pc, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double mx = -INFINITY;
  for (double v : lw) mx = std::max(mx, v);
  if (mx == -INFINITY) {
    *log_r = -INFINITY;
  } else {
    double W = 0.0;
    for (double v : lw) W += exp(v - mx);
    *log_r = lpc + mx + log(W / (double)c->nw);
  }
  return 0;
}

extern "C" int lecqmc_cp_walker(lecqmc_cp *c, int32_t a, double *log_w, double *log_q, int8_t *fields) {
  if (!c || a < 0 || a >= c->nw) return fail(LECQMC_EINVAL, "bad walker index");
  lecqmc_ctx *ctx = c->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  if (log_w) HIPCHK(xfer(ctx, log_w, c->d.cur.logw + a, sizeof(double), hipMemcpyDeviceToHost));
  if (log_q) HIPCHK(xfer(ctx, log_q, c->d.cur.logq + a, sizeof(double), hipMemcpyDeviceToHost));
  if (fields)
    HIPCHK(xfer(ctx, fields, c->d.cur.s + (size_t)a * c->L * c->N, (size_t)c->L * c->N, hipMemcpyDeviceToHost));
  return 0;
}

extern "C" int lecqmc_cp_stats(lecqmc_cp *c, double *log_pc, int64_t *cuts, int32_t *alive) {
  if (!c) return fail(LECQMC_EINVAL, "null argument");
  lecqmc_ctx *ctx = c->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<double> lw(c->nw);
  std::vector<long long> cu(c->nw);
  double lpc = 0.0;
  HIPCHK(xfer(ctx, lw.data(), c->d.cur.logw, sizeof(double) * c->nw, hipMemcpyDeviceToHost));
  HIPCHK(xfer(ctx, cu.data(), c->d.cuts, sizeof(long long) * c->nw, hipMemcpyDeviceToHost));
  HIPCHK(xfer(ctx, &lpc, c->d.log_pc, sizeof(double), hipMemcpyDeviceToHost));
  if (log_pc) *log_pc = lpc;
  if (cuts) {
    long long s = 0;
    for (long long v : cu) s += v;
    *cuts = s;
  }
  if (alive) {
    int n = 0;
    for (double v : lw) n += v > -INFINITY;
    *alive = n;
  }
  return 0;
}

extern "C" int lecqmc_cp_destroy(lecqmc_cp *c) {
  if (!c) return 0;
  (void)hipSetDevice(c->ctx->device);
  (void)hipStreamSynchronize(c->ctx->stream);
  (void)hipFree(c->dmem);
  c->ctx->used -= c->bytes;
  lecqmc_destroy_walker(c->trial);
  delete c;
  return 0;
}
