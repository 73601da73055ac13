// gfx950 kernels of the canonical-ensemble DQMC hot path.
//
// One workgroup of 256 threads (4 wave64) owns one walker (or one spin of a
// walker) for the whole of a phase; a batch launch gives every walker its own
// workgroup(s), so walkers of different shapes share one launch.  In the
// forward pass the right Slater blocks Phi_R (N x Ne, row-major) stay in LDS
// when they fit, and the left blocks are streamed from device memory in
// staged chunks of sites.  One wave runs the sequential Ising-flip chain,
// both spin species in the two halves of the wave: for Ne <= 32 the Ne x Ne
// inverses (P^T B P)^{-1} are held in that wave's registers, above that in
// LDS or device memory with delayed (Woodbury) updates on the FP64 matrix
// cores.  The other three waves stage the next chunk meanwhile.
//
// Method (arXiv 2601.08552): weight of main text Eq. (1); HS-field updates
// with the rank-1 fast update of the PQMC-like sweep (main text, "Ensemble
// constrained QMC"); QR stabilisation every tau_w slices and the stabilized
// QR update for particle removal / addition (SM Sec. I.A and I.B).
#include <math.h>

#include <mutex>
#include <type_traits>

#include "lecqmc_internal.h"

namespace lecqmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplies by 0xD2511F53 / 0xCD9E8D57 with the Weyl key
// schedule 0x9E3779B9 / 0xBB67AE85.  Counter (a, b, sweep, stream | id << 8),
// key = seed; the double is the top 53 bits of (out0:out1) times 2^-53.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t wid, uint32_t stream,
                                            uint32_t sweep, uint32_t a, uint32_t b) {
  uint32_t x0 = a, x1 = b, x2 = sweep, x3 = (stream & 0xffu) | (uint32_t)((wid & 0xffffffull) << 8);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  const uint64_t bits = ((uint64_t)x0 << 32) | x1;
  return (double)(bits >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ int pick(double u, int n) {
  int v = (int)floor(u * (double)n);
  return v >= n ? n - 1 : v;
}

// ---------------------------------------------------------------------------
// LDS layout (dynamic): sized by the largest Ne of the launch (mm) and by the
// Slater blocks kept resident in LDS (phi_elems doubles, 0 = streamed from
// device memory through the staging buffers).
// ---------------------------------------------------------------------------
struct Lds {
  double *red;    // 256   block reductions
  double *scal;   // 64    broadcast scalars
  int *iscal;     // 320   broadcast integers + per-thread counts
  double *Ms0;    // mm^2  inverse, spin up   (Fock phase: Hessenberg work)
  double *Ms1;    // mm^2  inverse, spin down (Fock phase: permuted inverse)
  double *A;      // mm^2  Gram / Cholesky / pivot work (Fock phase: reduced inverse)
  double *B;      // mm^2  triangular inverse / output
  double *vec;    // 8*vs  small vectors
  double *uw;     // 4*vs  u and w of an accepted site per spin (LDS-inverse chain)
  double *xs;     // [2 buf][2 spin][S][xld] staged left rows
  double *ps;     // [2 buf][2 spin][S][xld] staged right rows (streamed mode)
  double *us;     // [2 buf][S]              staged uniforms
  double *dl;     // [2 buf][2 spin][S]      staged flip factors Delta
  int8_t *fs;     // [2 buf][S]              staged Ising fields
  double *dg;     // delayed chains: chunk and coefficient matrices (dgn doubles), or nullptr
  int dgn;
  double *phi;    // resident Slater blocks, or nullptr
  double *bonds;  // compact bond tables (coef | bij | bci), or nullptr
  int S;          // sites per staged chunk
  bool bonds_ok;  // the walker's bond tables were copied into LDS
  int *cs;        // colour offsets copied into LDS (iscal + 16), or nullptr
  int vs;         // length of each small vector: max(64, largest Ne of the launch)
};

__host__ __device__ inline int vec_len(int mm) { return mm > 64 ? mm : 64; }
__host__ __device__ inline size_t lds_doubles_fixed(const LdsPlan &p) {
  const size_t mm = p.mm < 1 ? 1 : p.mm, S = p.smax > 0 ? p.smax : 0, vs = vec_len((int)mm);
  const size_t mats = (p.gm == 1 ? 0 : p.gm == 3 ? 1 : p.gm == 2 ? 2 : 4) * mm * mm;
  return 256 + 64 + mats + 8 * vs + 4 * vs + (p.stage_ps ? 2 : 1) * (size_t)p.xs_elems + 2 * S +
         4 * S + (2 * S + 7) / 8 + (size_t)p.dgn;
}

size_t lds_bytes(const LdsPlan &p) {
  const size_t d = lds_doubles_fixed(p) + (size_t)p.phi_elems + ((size_t)p.bond_words + 1) / 2;
  return d * sizeof(double) + 320 * sizeof(int);
}

extern __shared__ double lds_raw[];

// LEAN: the plan is known to keep all four work matrices in LDS and to have
// no delayed-chain area (launches of register-tiled walkers), which keeps
// fewer values live in the kernels that use it.
template <bool LEAN = false>
__device__ __forceinline__ Lds carve(const LdsPlan &pl) {
  const int mm = pl.mm < 1 ? 1 : pl.mm;
  const int S = pl.smax > 0 ? pl.smax : 0;
  Lds L;
  double *p = lds_raw;
  const int vs = LEAN ? 64 : vec_len(mm);
  L.red = p; p += 256;
  L.scal = p; p += 64;
  L.Ms0 = L.Ms1 = L.A = L.B = nullptr;   // those not in LDS are bound per walker by bind_mats
  if (LEAN || pl.gm == 0 || pl.gm == 2) {
    L.Ms0 = p; p += mm * mm;
    L.Ms1 = p; p += mm * mm;
  } else if (pl.gm == 3) {
    L.Ms0 = p; p += mm * mm;
  }
  if (LEAN || pl.gm == 0) {
    L.A = p; p += mm * mm;
    L.B = p; p += mm * mm;
  }
  L.vs = vs;
  L.vec = p; p += 8 * vs;
  L.uw = p; p += 4 * vs;
  L.xs = p; p += pl.xs_elems;
  L.ps = pl.stage_ps ? p : nullptr; p += pl.stage_ps ? pl.xs_elems : 0;
  L.us = p; p += 2 * S;
  L.dl = p; p += 4 * S;
  L.fs = reinterpret_cast<int8_t *>(p); p += (2 * S + 7) / 8;
  if (LEAN) {
    L.dg = nullptr;
    L.dgn = 0;
  } else {
    L.dg = pl.dgn > 0 ? p : nullptr;
    L.dgn = pl.dgn;
    p += pl.dgn;
  }
  L.phi = pl.phi_elems > 0 ? p : nullptr; p += pl.phi_elems;
  L.bonds = pl.bond_words > 0 ? p : nullptr; p += (pl.bond_words + 1) / 2;
  L.iscal = reinterpret_cast<int *>(p);
  L.S = S;
  L.bonds_ok = false;
  L.cs = nullptr;
  return L;
}
// Ne x Ne work matrices in device memory (plans with gm = 1: all four; gm =
// 2: the scratch pair A, B; gm = 3, the Fock phase only: all but the first):
// slot 0 for kernels with one workgroup per walker, the spin for those with
// one per (walker, spin).  The matrices are addressed with the walker's own Ne.
__device__ __forceinline__ void bind_mats(Lds &L, const WalkerDesc &w, const LdsPlan &pl, int slot) {
  if (pl.gm == 0) return;
  const size_t q = (size_t)w.mmax * w.mmax;
  double *base = w.bigm + (size_t)slot * 4 * q;
  if (pl.gm == 1) L.Ms0 = base;
  if (pl.gm == 1 || pl.gm == 3) L.Ms1 = base + q;
  L.A = base + 2 * q;
  L.B = base + 3 * q;
}
__device__ __forceinline__ LdsPlan parity_plan(int mm) { return LdsPlan{mm, 0, 1, 0, 0, 0, mm > kLdsNe ? 1 : 0, 0}; }

#define TID (static_cast<int>(threadIdx.x))
#define SYNC() __syncthreads()

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full barrier waits for every outstanding load).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ double wg_sum(double v, double *red) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  SYNC();
  if ((TID & 63) == 0) red[TID >> 6] = v;
  SYNC();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ double wg_max(double v, double *red) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  SYNC();
  if ((TID & 63) == 0) red[TID >> 6] = v;
  SYNC();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ---------------------------------------------------------------------------
// Propagation of N x m blocks (rows = sites): checkerboard colour passes and
// the diagonal Ising/onsite factor.  Each pass is written once for blocks in
// device memory and once for blocks resident in LDS (address-space-typed
// pointers, so the bond-table loads are not ordered behind LDS stores).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) int8_t lds_i8;
__device__ __forceinline__ lds_f64 *as_lds(double *p) { return (lds_f64 *)p; }
__device__ __forceinline__ lds_f32 *as_lds(float *p) { return (lds_f32 *)p; }
// barrier after a pass over X: LDS-only when X lives in LDS
template <typename P> struct PassSync { __device__ static void run() { SYNC(); } };
template <> struct PassSync<lds_f64 *> { __device__ static void run() { lds_sync(); } };
template <> struct PassSync<lds_f32 *> { __device__ static void run() { lds_sync(); } };
// arithmetic type of a pass over storage P: FP32 storage is propagated in FP32
template <typename P> struct Elem { using T = double; };
template <> struct Elem<float *> { using T = float; };
template <> struct Elem<lds_f32 *> { using T = float; };
__device__ __forceinline__ const lds_f64 *as_lds(const double *p) { return (const lds_f64 *)p; }
__device__ __forceinline__ const lds_f32 *as_lds(const float *p) { return (const lds_f32 *)p; }
__device__ __forceinline__ lds_i8 *as_lds(int8_t *p) { return (lds_i8 *)p; }

typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// One v_mfma_f64_16x16x4f64 (FP64 matrix cores).  Operand layouts (lane l,
// c = l % 16, g = l / 16): A (16 x 4) holds A[c][g], B (4 x 16) holds
// B[g][c], and element j of the 16 x 16 result holds D[4 j + g][c].
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// bond (i, j, cosh, -sinh) of bond b: from the compact LDS tables when they
// were loaded, from device memory otherwise
struct BondSrc {
  const lds_f64 *coef;
  const lds_i32 *bij;
  const lds_u8 *bci;
  const lds_i32 *cs;  // colour offsets in LDS, or nullptr
  bool lds;
};
__device__ __forceinline__ BondSrc bond_src(const Lds &L, const WalkerDesc &w) {
  BondSrc b;
  b.lds = L.bonds_ok;
  b.cs = L.cs ? (const lds_i32 *)L.cs : nullptr;
  double *base = L.bonds ? L.bonds : L.red;
  b.coef = as_lds(base);
  b.bij = (const lds_i32 *)(as_lds(base) + 2 * kMaxCoef);
  b.bci = (const lds_u8 *)(b.bij + w.nbonds);
  return b;
}
template <bool TL>
__device__ __forceinline__ void bond_get_t(const WalkerDesc &w, const BondSrc &bs, int b, int &i, int &j, double &d,
                                           double &o) {
  if constexpr (TL) {
    const int ij = bs.bij[b];
    i = ij & 0xffff;
    j = (int)((unsigned)ij >> 16);
    const int ci = bs.bci[b];
    d = bs.coef[2 * ci];
    o = bs.coef[2 * ci + 1];
  } else {
    i = w.bi[b];
    j = w.bj[b];
    d = w.bdiag[b];
    o = w.boff[b];
  }
}
__device__ __forceinline__ void bond_get(const WalkerDesc &w, const BondSrc &bs, int b, int &i, int &j, double &d,
                                         double &o) {
  if (bs.lds) {
    const int ij = bs.bij[b];
    i = ij & 0xffff;
    j = (int)((unsigned)ij >> 16);
    const int ci = bs.bci[b];
    d = bs.coef[2 * ci];
    o = bs.coef[2 * ci + 1];
  } else {
    i = w.bi[b];
    j = w.bj[b];
    d = w.bdiag[b];
    o = w.boff[b];
  }
}

// copy the compact bond tables of walker w into LDS (all threads)
// copy the compact bond tables of walker w into LDS, and the colour offsets
// (read at every colour pass) when there are at most 47 colours (all threads)
__device__ __forceinline__ void load_bonds(const WalkerDesc &w, Lds &L, int plan_words) {
  if (w.ncol + 1 <= 48) {
    for (int t = TID; t <= w.ncol; t += kThreads) L.iscal[16 + t] = w.col_start[t];
    L.cs = L.iscal + 16;
  }
  L.bonds_ok = L.bonds != nullptr && w.ncoef > 0 && w.bond_words <= plan_words;
  if (L.bonds_ok) {
    lds_f64 *coef = as_lds(L.bonds);
    lds_i32 *bij = (lds_i32 *)(coef + 2 * kMaxCoef);
    lds_u8 *bci = (lds_u8 *)(bij + w.nbonds);
    for (int t = TID; t < 2 * w.ncoef; t += kThreads) coef[t] = w.coef[t];
    for (int t = TID; t < w.nbonds; t += kThreads) {
      bij[t] = w.bij[t];
      bci[t] = w.bci[t];
    }
  }
  SYNC();
}
__device__ __forceinline__ int colour_begin(const WalkerDesc &w, const BondSrc &bs, int c) {
  return bs.cs ? bs.cs[c] : w.col_start[c];
}

template <bool TL, typename P>
__device__ __forceinline__ void colour_pass_tt(const WalkerDesc &w, const BondSrc &bs, P X, int m, int b0, int b1,
                                               bool inverse) {
  using E = typename Elem<P>::T;
  // thread = (bond slot, column): column fastest, so neighbouring lanes touch
  // neighbouring words of a row; one division per pass, 32-bit indices
  const int per = m > 0 ? kThreads / m : 0;
  const int col = m > 0 ? TID % m : 0, slot = m > 0 ? TID / m : kThreads;
  if (slot < per) {
    // eight bonds per thread per round: all loads first, then all stores (the
    // bonds of one colour are disjoint, so nothing aliases).  A slot past the
    // colour's end loads bond b0 again and stores nothing, so that no load
    // waits behind a branch.
    constexpr int kB = 8;
    for (int bb = b0 + slot; bb < b1; bb += kB * per) {
      int ii[kB], jj[kB];
      E xi[kB], xj[kB], d[kB], o[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int b = bb + u * per < b1 ? bb + u * per : b0;
        int i, j;
        double dd, oo;
        bond_get_t<TL>(w, bs, b, i, j, dd, oo);
        d[u] = (E)dd;
        o[u] = (E)(inverse ? -oo : oo);
        ii[u] = i * m + col;
        jj[u] = j * m + col;
        xi[u] = X[ii[u]];
        xj[u] = X[jj[u]];
      }
#pragma unroll
      for (int u = 0; u < kB; ++u)
        if (bb + u * per < b1) {
          X[ii[u]] = d[u] * xi[u] + o[u] * xj[u];
          X[jj[u]] = o[u] * xi[u] + d[u] * xj[u];
        }
    }
  }
  PassSync<P>::run();
}
template <typename P>
__device__ __forceinline__ void colour_pass_t(const WalkerDesc &w, const BondSrc &bs, P X, int m, int c,
                                              bool inverse) {
  const int b0 = colour_begin(w, bs, c), b1 = colour_begin(w, bs, c + 1);
  if (bs.lds) colour_pass_tt<true>(w, bs, X, m, b0, b1, inverse);
  else colour_pass_tt<false>(w, bs, X, m, b0, b1, inverse);
}

template <typename P>
__device__ __forceinline__ void diag_t(const WalkerDesc &w, P X, int m, int l, int sp, bool inverse) {
  using E = typename Elem<P>::T;
  const int N = w.N;
  const int8_t *s = w.s + (size_t)(l - 1) * N;
  const double elam = w.elam, emlam = w.emlam;
  // the fields and onsite factors of four rows are loaded before any row is scaled
  constexpr int R = 4;
  for (int i0 = TID; i0 < N; i0 += R * kThreads) {
    int sv[R];
    double ev[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r * kThreads;
      sv[r] = i < N ? s[i] : 1;
      ev[r] = i < N ? w.eps_fac[i] : 1.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r * kThreads;
      if (i < N) {
        const int ss = sp == 0 ? sv[r] : -sv[r];
        double f = (ss > 0 ? elam : emlam) * ev[r];
        if (inverse) f = 1.0 / f;
        const E fe = (E)f;
        for (int a = 0; a < m; ++a) X[(size_t)i * m + a] *= fe;
      }
    }
  }
  PassSync<P>::run();
}

__device__ __forceinline__ bool in_lds(const void *p) {
  return __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void *)p);
}

template <typename F>
__device__ void colour_pass(const WalkerDesc &w, const Lds &L, F *X, int m, int c, bool inverse) {
  const BondSrc bs = bond_src(L, w);
  if (in_lds(X)) colour_pass_t(w, bs, as_lds(X), m, c, inverse);
  else colour_pass_t(w, bs, X, m, c, inverse);
}
// X <- E_K X : colour C-1 acts first
template <typename F>
__device__ void apply_ek(const WalkerDesc &w, const Lds &L, F *X, int m) {
  for (int c = w.ncol - 1; c >= 0; --c) colour_pass(w, L, X, m, c, false);
}
// X <- E_K^T X : colour 0 acts first
template <typename F>
__device__ void apply_ekT(const WalkerDesc &w, const Lds &L, F *X, int m) {
  for (int c = 0; c < w.ncol; ++c) colour_pass(w, L, X, m, c, false);
}
// X <- D_l^{+-1} X for spin sp (l = 1..L)
template <typename F>
__device__ __noinline__ void apply_diag(const WalkerDesc &w, F *X, int m, int l, int sp, bool inverse) {
  if (in_lds(X)) diag_t(w, as_lds(X), m, l, sp, inverse);
  else diag_t(w, X, m, l, sp, inverse);
}

template <typename F>
__device__ void fill_P(const WalkerDesc &w, int sp, F *X) {
  const int m = w.ne[sp], tot = w.N * m;
  for (int t = TID; t < tot; t += kThreads) X[t] = (F)0;
  SYNC();
  for (int a = TID; a < m; a += kThreads) X[(size_t)w.occ[sp][a] * m + a] = (F)1;
  SYNC();
}

// dst[0..n) = src[0..n); eight loads are issued before their stores, since
// the compiler cannot tell that dst and src do not overlap
template <typename D, typename S>
__device__ void copy_global(D *dst, const S *src, size_t n) {
  constexpr int U = 8;
  for (size_t t0 = TID; t0 < n; t0 += (size_t)U * kThreads) {
    D v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t t = t0 + (size_t)u * kThreads;
      v[u] = t < n ? (D)src[t] : (D)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t t = t0 + (size_t)u * kThreads;
      if (t < n) dst[t] = v[u];
    }
  }
  SYNC();
}

// partial sum_i X[i][pa] Y[i][qb] over rows i = i0, i0 + G, ... (optionally
// only rows with sub[i] == sa), four independent accumulators so that the
// loads of consecutive rows overlap
template <typename PX, typename PY>
__device__ __forceinline__ double gram_rows(PX X, int mx, int pa, PY Y, int my, int qb, int i0, int N, int G,
                                            const int *sub, int sa) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = i0;
  if (!sub) {
#pragma unroll 2
    for (; i + 3 * G < N; i += 4 * G) {
      a0 += (double)X[(size_t)i * mx + pa] * (double)Y[(size_t)i * my + qb];
      a1 += (double)X[(size_t)(i + G) * mx + pa] * (double)Y[(size_t)(i + G) * my + qb];
      a2 += (double)X[(size_t)(i + 2 * G) * mx + pa] * (double)Y[(size_t)(i + 2 * G) * my + qb];
      a3 += (double)X[(size_t)(i + 3 * G) * mx + pa] * (double)Y[(size_t)(i + 3 * G) * my + qb];
    }
    for (; i < N; i += G) a0 += (double)X[(size_t)i * mx + pa] * (double)Y[(size_t)i * my + qb];
  } else {
    for (; i < N; i += G)
      if (sub[i] == sa) a0 += (double)X[(size_t)i * mx + pa] * (double)Y[(size_t)i * my + qb];
  }
  return (a0 + a1) + (a2 + a3);
}

// out = X^T Y on the FP64 matrix cores, for Gram matrices larger than one
// entry per thread: 16 x 16 output tiles, four rows per step (A = X^T and
// B = Y: lane (c, g) loads X[i + g][p0 + c] and Y[i + g][q0 + c]; columns and
// rows past the ends load a clamped address and contribute zero).  A wave
// owns groups of up to four tiles that share one p tile (one A load per
// step).  With fewer groups than waves the rows are split among the waves
// and the partial tiles are added into out in a fixed wave order, so the
// result does not depend on timing.
template <typename PX, typename PY>
__device__ void gram_mfma(PX X, int mx, PY Y, int my, int N, double *out) {
  const int tp = (mx + 15) >> 4, tq = (my + 15) >> 4;
  const int qg = tq < 4 ? tq : 4;            // tiles per group
  const int gq = (tq + qg - 1) / qg;         // groups per p tile
  const int ng = tp * gq;
  const int ks = ng >= 4 ? 1 : 4 / ng;       // row splits (ng * ks <= 4 when ks > 1)
  const int wave = TID >> 6, lane = TID & 63, c = lane & 15, g = lane >> 4;
  const int steps = (N + 3) >> 2;
  for (int it = wave; it < ng * ks; it += 4) {
    const int grp = it % ng, part = it / ng;
    const int pt = grp / gq, qt0 = (grp - pt * gq) * qg;
    const int nq = min(qg, tq - qt0);
    const int s0 = (int)((long)steps * part / ks), s1 = (int)((long)steps * (part + 1) / ks);
    const int pc = pt * 16 + c;
    const bool pv = pc < mx;
    const int pcc = pv ? pc : mx - 1;
    int qcc[4];
    bool qv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = (qt0 + j) * 16 + c;
      qv[j] = j < nq && q < my;
      qcc[j] = qv[j] ? q : my - 1;
    }
    v4d acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int st = s0; st < s1; ++st) {
      const int i = 4 * st + g;
      const bool iv = i < N;
      const int ic = iv ? i : N - 1;
      const double xa = (double)X[(size_t)ic * mx + pcc];
      double yb[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) yb[j] = (double)Y[(size_t)ic * my + qcc[j]];
      const double a = (iv && pv) ? xa : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nq) acc[j] = mfma_f64(a, (iv && qv[j]) ? yb[j] : 0.0, acc[j]);
    }
    // ks == 1: every tile is computed by one wave; ks > 1 only when
    // ng * ks == 4 (one item per wave, so every wave meets the same
    // barriers): the wave holding row part `part` adds its tiles in phase part
    for (int ph = 0; ph < ks; ++ph) {
      if (ph == part) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nq && qv[j])
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int p = pt * 16 + 4 * r + g;
              if (p < mx) {
                double &o = out[p * my + (qt0 + j) * 16 + c];
                o = ph == 0 ? acc[j][r] : o + acc[j][r];
              }
            }
      }
      if (ks > 1) SYNC();
    }
  }
  SYNC();
}

template <typename PX, typename PY>
__device__ void gram_t(PX X, int mx, PY Y, int my, int N, double *out, double *red, const int *sub, int sa) {
  const int P = mx * my;
  if (P > kThreads && !sub) {
    gram_mfma(X, mx, Y, my, N, out);
  } else if (P <= kThreads) {
    const int G = kThreads / P;
    const int g = TID / P, p = TID - g * P;
    double acc = 0.0;
    if (g < G) {
      const int pa = p / my, qb = p - pa * my;
      acc = gram_rows(X, mx, pa, Y, my, qb, g, N, G, sub, sa);
    }
    SYNC();
    red[TID] = acc;
    SYNC();
    if (TID < P) {
      double s = 0.0;
      for (int gg = 0; gg < G; ++gg) s += red[gg * P + TID];
      out[TID] = s;
    }
    SYNC();
  } else {
    for (int p = TID; p < P; p += kThreads) {
      const int pa = p / my, qb = p - pa * my;
      out[p] = gram_rows(X, mx, pa, Y, my, qb, 0, N, 1, sub, sa);
    }
    SYNC();
  }
}

// out[p][q] = sum_i X[i][p] Y[i][q] over rows i (optionally only sub[i] == a),
// accumulated in FP64 for FP32 or FP64 storage
template <typename TX, typename TY>
__device__ void gram(const TX *X, int mx, const TY *Y, int my, int N, double *out,
                     double *red, const int *sub = nullptr, int sa = 0) {
  if (mx * my == 0) { SYNC(); return; }
  const bool lx = in_lds(X), ly = in_lds(Y);
  if (lx && ly) gram_t(as_lds(X), mx, as_lds(Y), my, N, out, red, sub, sa);
  else if (lx) gram_t(as_lds(X), mx, Y, my, N, out, red, sub, sa);
  else if (ly) gram_t(X, mx, as_lds(Y), my, N, out, red, sub, sa);
  else gram_t(X, mx, Y, my, N, out, red, sub, sa);
}

// Cholesky G = R^T R in place (upper triangle of A); false on a non-positive pivot.
__device__ bool cholesky(double *A, int m, double *scal) {
  for (int j = 0; j < m; ++j) {
    if (TID == 0) {
      const double d = A[j * m + j];
      scal[0] = d;
      A[j * m + j] = d > 0.0 ? sqrt(d) : d;
    }
    SYNC();
    if (!(scal[0] > 0.0)) { SYNC(); return false; }
    const double r = A[j * m + j];
    for (int c = j + 1 + TID; c < m; c += kThreads) A[j * m + c] /= r;
    SYNC();
    // trailing update, eight elements per thread and round with every load
    // before any store (row j is not written here); one element per thread
    // when they all fit in one round
    const int rem = m - j - 1, tot = rem * rem;
    if (tot <= kThreads) {
      if (TID < tot) {
        const int a = j + 1 + TID / rem, c = j + 1 + TID % rem;
        if (c >= a) A[a * m + c] -= A[j * m + a] * A[j * m + c];
      }
      SYNC();
      continue;
    }
    for (int t0 = TID; t0 < tot; t0 += 8 * kThreads) {
      double x[8], ra[8], rc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * kThreads, tc = t < tot ? t : 0;
        const int a = j + 1 + tc / rem, c = j + 1 + tc % rem;
        x[u] = A[a * m + c];
        ra[u] = A[j * m + a];
        rc[u] = A[j * m + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * kThreads;
        const int a = j + 1 + t / (rem > 0 ? rem : 1), c = j + 1 + t % (rem > 0 ? rem : 1);
        if (t < tot && c >= a) A[a * m + c] = x[u] - ra[u] * rc[u];
      }
    }
    SYNC();
  }
  return true;
}

// sum_{b = b0 .. b1} A[b] * B[b * sb], accumulated in order b0, b0 + 1, ...;
// the operands of eight terms are loaded before they are added, so that the
// loads of a matrix in device memory overlap
__device__ __forceinline__ double dot_in_order(const double *A, const double *B, int sb, int b0, int b1) {
  double s = 0.0;
  int b = b0;
  for (; b + 7 <= b1; b += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] = A[b + u];
      y[u] = B[(size_t)(b + u) * sb];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u] * y[u];
  }
  for (; b <= b1; ++b) s += A[b] * B[(size_t)b * sb];
  return s;
}

// Ri = R^{-1} (upper triangular), column by column
__device__ void tri_inverse(const double *R, int m, double *Ri) {
  for (int c = TID; c < m; c += kThreads) {
    for (int a = c + 1; a < m; ++a) Ri[a * m + c] = 0.0;
    Ri[c * m + c] = 1.0 / R[c * m + c];
    for (int a = c - 1; a >= 0; --a) {
      const double s = dot_in_order(R + a * m, Ri + c, m, a + 1, c);
      Ri[a * m + c] = -s / R[a * m + a];
    }
  }
  SYNC();
}

// out = in * Ri (Ri upper triangular, m x m) on the FP64 matrix cores,
// m > 8: one 16-row strip per wave at a time, output tiles of 16 columns
// from the last to the first.  Tile t (columns 16 t .. 16 t + 15) reads only
// the strip's columns below 16 t + 16 (Ri[k][q] = 0 for k > q) and those have
// not been stored yet, so in and out may be the same block (lane (c, g)
// loads in[i0 + c][4 k + g] as the A operand).  The result also goes to out2
// (if set).
template <typename PI, typename PO>
__device__ void trimul_mfma(PI in, PO out, double *out2, int N, int m, const double *Ri) {
  const int wave = TID >> 6, lane = TID & 63, c = lane & 15, g = lane >> 4;
  const int nks = (m + 3) >> 2, tq = (m + 15) >> 4;
  const double *R = Ri;   // LDS, or device memory when the launch keeps its Ne x Ne matrices there
  for (int st = wave; st * 16 < N; st += 4) {
    const int i = st * 16 + c;
    const bool iv = i < N;
    const int ic = iv ? i : N - 1;
    for (int t = tq - 1; t >= 0; --t) {
      const int q = t * 16 + c;
      const bool qv = q < m;
      const int qc = qv ? q : m - 1;
      const int kend = min(nks, 4 * t + 4);
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
      for (int k = 0; k < kend; ++k) {
        const int kk = 4 * k + g;
        const bool kv = kk < m;
        const int kc = kv ? kk : m - 1;
        const double a = (double)in[(size_t)ic * m + kc];
        const double b = R[kc * m + qc];
        acc = mfma_f64((iv && kv) ? a : 0.0, (kv && qv) ? b : 0.0, acc);
      }
      if (qv)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = st * 16 + 4 * r + g;
          if (row < N) {
            out[(size_t)row * m + q] = acc[r];
            if (out2) out2[(size_t)row * m + q] = acc[r];
          }
        }
    }
  }
}

// out = in * Ri (Ri upper triangular), written to out and out2 (if set)
template <typename TI>
__device__ void right_tri_mul(const TI *in, double *out, double *out2, int N, int m, const double *Ri) {
  if (m > 8) {
    if (in_lds(in)) {
      if (in_lds(out)) trimul_mfma(as_lds(in), as_lds(out), out2, N, m, Ri);
      else trimul_mfma(as_lds(in), out, out2, N, m, Ri);
    } else {
      if (in_lds(out)) trimul_mfma(in, as_lds(out), out2, N, m, Ri);
      else trimul_mfma(in, out, out2, N, m, Ri);
    }
    SYNC();
    return;
  }
  const int tot = N * m;
  for (int t = TID; t < tot; t += kThreads) {
    const int i = t / m, c = t - (t / m) * m;
    const TI *row = in + (size_t)i * m;
    double s = 0.0;
    for (int a = 0; a <= c; ++a) s += (double)row[a] * Ri[a * m + c];
    out[t] = s;
    if (out2) out2[t] = s;
  }
  SYNC();
}

// X <- X * Ri in place (Ri upper triangular), one thread per row: row i of
// the product needs only row i of X.  A row of at most MR entries is held in
// registers; a longer one is rewritten from its last column to its first, so
// that column c still reads the unmodified entries 0..c.  Each entry is
// summed in the order right_tri_mul uses.  The result also goes to out2 (if
// set).
template <int MR, typename P>
__device__ __forceinline__ void tri_mul_rows_t(P X, double *out2, int N, int m, const double *Ri) {
  for (int i = TID; i < N; i += kThreads) {
    P row = X + (size_t)i * m;
    double *o2 = out2 ? out2 + (size_t)i * m : nullptr;
    if (m <= MR) {
      double r[MR];
#pragma unroll
      for (int a = 0; a < MR; ++a) r[a] = a < m ? (double)row[a] : 0.0;
#pragma unroll
      for (int c = 0; c < MR; ++c) {
        if (c < m) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a <= c; ++a) s += r[a] * Ri[a * m + c];
          row[c] = s;
          if (o2) o2[c] = s;
        }
      }
    } else {
      for (int c = m - 1; c >= 0; --c) {
        double s = 0.0;
        for (int a = 0; a <= c; ++a) s += (double)row[a] * Ri[a * m + c];
        row[c] = s;
        if (o2) o2[c] = s;
      }
    }
  }
  SYNC();
}
template <int MR>
__device__ __forceinline__ void tri_mul_rows(double *X, double *out2, int N, int m, const double *Ri) {
  if (m > MR) {
    if (in_lds(X)) trimul_mfma(as_lds(X), as_lds(X), out2, N, m, Ri);
    else trimul_mfma(X, X, out2, N, m, Ri);
    SYNC();
    return;
  }
  if (in_lds(X)) tri_mul_rows_t<MR>(as_lds(X), out2, N, m, Ri);
  else tri_mul_rows_t<MR>(X, out2, N, m, Ri);
}

// CholeskyQR2 of an FP64 block in its own storage: X (N x m) -> Q, also
// stored to out2 (if set).  Returns false, with X untouched, when the first
// Gram matrix is not numerically positive definite.  Same arithmetic as the
// general path below, without its device-memory intermediates.
template <int MR>
__device__ bool cholqr_inplace(double *X, double *out2, double *Vout, double *Vacc, int N, int m, Lds &L,
                               Scalars *sc, double *ld) {
  gram(X, m, X, m, N, L.A, L.red);
  if (!cholesky(L.A, m, L.scal)) return false;
  for (int t = TID; t < m * m; t += kThreads) {
    const int a = t / m, c = t % m;
    Vacc[t] = c >= a ? L.A[t] : 0.0;
  }
  tri_inverse(L.A, m, L.B);
  tri_mul_rows<MR>(X, nullptr, N, m, L.B);
  gram(X, m, X, m, N, L.A, L.red);
  if (!cholesky(L.A, m, L.scal)) {
    if (TID == 0) sc->status |= 4;
  }
  tri_inverse(L.A, m, L.B);
  tri_mul_rows<MR>(X, out2, N, m, L.B);
  for (int t = TID; t < m * m; t += kThreads) {
    const int a = t / m, c = t % m;
    const double s = c >= a ? dot_in_order(L.A + a * m, Vacc + c, m, a, c) : 0.0;
    L.B[t] = c >= a ? s : 0.0;
  }
  SYNC();
  for (int t = TID; t < m * m; t += kThreads) {
    Vacc[t] = L.B[t];
    if (Vout) Vout[t] = L.B[t];
  }
  SYNC();
  double s = 0.0;
  for (int a = 0; a < m; ++a) s += log(Vacc[a * m + a]);
  SYNC();
  *ld = s;
  return true;
}

// Thin QR with positive diagonal by Cholesky QR, repeated (CholeskyQR2;
// a shifted first pass and a third pass when the Gram matrix is not
// numerically positive definite).  Phi (N x m) -> Q in q1 (and q2); the
// triangular factor R = R_last ... R_1 goes to Vout (m x m, may be null).
// tmp: N x m scratch distinct from Phi, q1, q2.  Vacc: m x m global scratch.
// Returns sum_j log R_jj.
// Phi and q2 are FP64 or FP32 storage; the Gram matrices, factors and tmp,
// q1 are FP64.
// An FP64 block that is itself one of the outputs (q1 or q2) is factored in
// place (MR: longest row held in registers).
template <typename F, int MR = 8>
__device__ __forceinline__ double cholqr(const F *Phi, double *tmp, double *q1, F *q2, double *Vout,
                         double *Vacc, int N, int m, Lds &L, Scalars *sc) {
  if (m == 0) { SYNC(); return 0.0; }
  if constexpr (std::is_same<F, double>::value) {
    if (q1 == Phi || q2 == Phi) {
      double ld;
      if (cholqr_inplace<MR>(const_cast<double *>(Phi), q1 == Phi ? q2 : q1, Vout, Vacc, N, m, L, sc, &ld))
        return ld;
    }
  }
  bool shifted = false;
  // pass 1: Phi -> tmp
  gram(Phi, m, Phi, m, N, L.A, L.red);
  if (!cholesky(L.A, m, L.scal)) {
    gram(Phi, m, Phi, m, N, L.A, L.red);
    if (TID == 0) {
      double tr = 0.0;
      for (int a = 0; a < m; ++a) tr += L.A[a * m + a];
      const double shift = 11.0 * ((double)N * m + (double)m * (m + 1)) * 0x1.0p-53 * tr;
      for (int a = 0; a < m; ++a) L.A[a * m + a] += shift;
      sc->qr_shifted += 1;
      sc->status |= 2;
    }
    SYNC();
    cholesky(L.A, m, L.scal);
    shifted = true;
  }
  for (int t = TID; t < m * m; t += kThreads) {
    const int a = t / m, c = t % m;
    Vacc[t] = c >= a ? L.A[t] : 0.0;
  }
  tri_inverse(L.A, m, L.B);
  right_tri_mul(Phi, tmp, nullptr, N, m, L.B);
  const int passes = shifted ? 3 : 2;
  for (int pass = 1; pass < passes; ++pass) {
    const double *in = (pass == 1) ? tmp : q1;
    double *out = (pass == 1) ? q1 : tmp;
    gram(in, m, in, m, N, L.A, L.red);
    if (!cholesky(L.A, m, L.scal)) {
      if (TID == 0) sc->status |= 4;
    }
    tri_inverse(L.A, m, L.B);
    right_tri_mul(in, out, nullptr, N, m, L.B);
    // Vacc <- R_pass * Vacc (both upper triangular) via B
    for (int t = TID; t < m * m; t += kThreads) {
      const int a = t / m, c = t % m;
      const double s = c >= a ? dot_in_order(L.A + a * m, Vacc + c, m, a, c) : 0.0;
      L.B[t] = c >= a ? s : 0.0;
    }
    SYNC();
    for (int t = TID; t < m * m; t += kThreads) Vacc[t] = L.B[t];
    SYNC();
  }
  // final Q lives in q1 (2 passes) or tmp (3 passes)
  const double *qf = (passes == 2) ? q1 : tmp;
  const int tot = N * m;
  for (int t = TID; t < tot; t += kThreads) {
    const double v = qf[t];
    if (passes != 2) q1[t] = v;
    if (q2) q2[t] = (F)v;
  }
  if (Vout)
    for (int t = TID; t < m * m; t += kThreads) Vout[t] = Vacc[t];
  SYNC();
  double ld = 0.0;
  for (int a = 0; a < m; ++a) ld += log(Vacc[a * m + a]);
  SYNC();
  return ld;
}

// Inverse by Gauss-Jordan elimination with partial pivoting.
// M (LDS, m x m) is destroyed; Minv may be LDS or global.  log|det|, sign
// and a singular flag are returned through scal / iscal.
__device__ __noinline__ bool gj_inverse(double *M, double *Minv, int m, Lds &L, double *logabs, int *sign) {
  for (int t = TID; t < m * m; t += kThreads) Minv[t] = (t / m == t % m) ? 1.0 : 0.0;
  if (TID == 0) { L.scal[2] = 0.0; L.iscal[1] = 1; L.iscal[2] = 0; }
  SYNC();
  double *fac = L.vec + 7 * L.vs;
  for (int c = 0; c < m; ++c) {
    if (m <= 32) {
      // short columns: one thread scans them in order
      if (TID == 0) {
        int p = c;
        double best = fabs(M[c * m + c]);
        for (int r = c + 1; r < m; ++r)
          if (fabs(M[r * m + c]) > best) { best = fabs(M[r * m + c]); p = r; }
        L.iscal[0] = p;
        L.scal[1] = M[p * m + c];
        if (best == 0.0) L.iscal[2] = 1;
        if (p != c) L.iscal[1] = -L.iscal[1];
      }
    } else if (TID < 64) {
      // the first row (in row order) of largest |M[r][c]|, r >= c: each lane
      // scans rows c + lane, c + lane + 64, ... in order, then the wave keeps
      // the larger value and, on a tie, the lower row
      double best = -1.0;
      int p = m;
      for (int r = c + TID; r < m; r += 64) {
        const double v = fabs(M[r * m + c]);
        if (v > best) { best = v; p = r; }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int op = __shfl_xor(p, off);
        if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
      }
      if (TID == 0) {
        L.iscal[0] = p;
        L.scal[1] = M[p * m + c];
        if (best == 0.0) L.iscal[2] = 1;
        if (p != c) L.iscal[1] = -L.iscal[1];
      }
    }
    SYNC();
    if (L.iscal[2]) { SYNC(); *logabs = -INFINITY; *sign = 0; return false; }
    const int p = L.iscal[0];
    const double piv = L.scal[1];
    if (p != c) {
      for (int x = TID; x < m; x += kThreads) {
        double t0 = M[c * m + x]; M[c * m + x] = M[p * m + x]; M[p * m + x] = t0;
        double t1 = Minv[c * m + x]; Minv[c * m + x] = Minv[p * m + x]; Minv[p * m + x] = t1;
      }
      SYNC();
    }
    for (int x = TID; x < m; x += kThreads) { M[c * m + x] /= piv; Minv[c * m + x] /= piv; }
    if (TID == 0) {
      L.scal[2] += log(fabs(piv));
      if (piv < 0.0) L.iscal[1] = -L.iscal[1];
    }
    SYNC();
    for (int r = TID; r < m; r += kThreads) fac[r] = M[r * m + c];
    SYNC();
    // eight elements per thread and round: every load before any store
    // (no element of the pivot row is written in this step)
    const int tot = m * m;
    for (int t0 = TID; t0 < tot; t0 += 8 * kThreads) {
      double a[8], b[8], pa[8], pb[8], f[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * kThreads, tc = t < tot ? t : 0;
        const int r = tc / m, x = tc - r * m;
        a[u] = M[tc];
        b[u] = Minv[tc];
        pa[u] = M[c * m + x];
        pb[u] = Minv[c * m + x];
        f[u] = fac[r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * kThreads;
        if (t < tot && t / m != c) {
          M[t] = a[u] - f[u] * pa[u];
          Minv[t] = b[u] - f[u] * pb[u];
        }
      }
    }
    SYNC();
  }
  *logabs = L.scal[2];
  *sign = L.iscal[1];
  SYNC();
  return true;
}

// ---------------------------------------------------------------------------
// Cross-lane sums inside one 32-lane half of a wave64 (DPP and permlane).
// Lane h = 8 ar + bc of a half.  sum_bc adds over bc (xor 1, xor 2, then the
// other quad through the 8-lane half mirror); sum_ar adds over ar (xor 8 by a
// rotate of 8 inside the 16-lane row, then the two 16-lane rows of the half
// through permlane16_swap).  Every lane of a group ends with the bit-identical
// sum, so decisions taken from it are uniform.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  // every lane reads a valid source lane for the patterns used here, so the
  // old value is never kept and no copy of it is made
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swz16_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_ds_swizzle(hi, 0x401F), __builtin_amdgcn_ds_swizzle(lo, 0x401F));
}
__device__ __forceinline__ double sum_bc(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  return v;
}
__device__ __forceinline__ double sum_ar(double v) {
  v += dpp_d<0x128>(v);  // row_ror:8
  // permlane16_swap of a register with itself yields, in every lane, the
  // value of the even 16-lane row of its pair of rows and that of the odd row
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
// (value of lane l & 31, value of lane (l & 31) + 32) for every lane l
__device__ __forceinline__ double halves_product(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double lower = __hiloint2double((int)b[0], (int)a[0]);
  const double upper = __hiloint2double((int)b[1], (int)a[1]);
  return lower * upper;
}
// sum over all 64 lanes of a wave, the same bits in every lane (8 lanes,
// then the 32-lane half, then the two halves)
__device__ __forceinline__ double wave_sum_d(double v) {
  v = sum_ar(sum_bc(v));
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double lane_read(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Sequential Ising-flip chain over one staged chunk of sites (wave 0).
// Lanes 0..31 carry spin up, lanes 32..63 spin down.  Per site i:
//   a_s = Phi_R[i,:] M_s^{-1} Phi_L[:,i],  r_s = 1 + Delta_s a_s,  r = r_up r_dn,
// accept if U(FLIP, sweep, l, i) < |r|; on acceptance the Sherman-Morrison
// update M^{-1} -= (Delta/r)(M^{-1} Phi_L[:,i])(Phi_R[i,:] M^{-1}) and the row
// scaling Phi_R[i,:] *= 1 + Delta (main text: fast update of the
// auxiliary-field sweep, as in projector QMC).
//
// Register-tiled version for Ne <= 8T: lane (ar, bc) of a half holds rows
// ar*2T .. ar*2T+2T-1 and columns bc*T .. bc*T+T-1 of its spin's inverse,
// in the lane-dependent slot order of tile_key / tile_ckey below.
// ---------------------------------------------------------------------------
// log|W| bookkeeping of accepted flips: a mantissa product renormalised by
// exponent bits (exact power-of-two scaling), logged once per block.
struct ChainAcc {
  double logw;
  double prod;
  int expo;
  long long nacc;
  int nnear;   // decisions whose uniform lies within kNearTie of |r|
};
// A decision u < |r| is counted as a near tie when |u - |r|| < kNearTie: a
// rounding difference in r that large could have reversed it.
constexpr double kNearTie = 1e-9;
__device__ __forceinline__ int near_tie_lane(double u, double absr) { return fabs(u - absr) < kNearTie ? 1 : 0; }
// In the chain wave u and |r| are the same in every lane: the tests go to
// wave masks, so that the decision and the count stay scalar.
__device__ __forceinline__ int near_tie(double u, double absr) {
  return __ballot(fabs(u - absr) < kNearTie) != 0ull ? 1 : 0;
}
__device__ __forceinline__ bool accept_site(double u, double absr) { return __ballot(u < absr) != 0ull; }
// prod stays in [1/2, 1): the exponent of every product is moved into expo
__device__ __forceinline__ void acc_ratio(ChainAcc &acc, double r) {
  const double pr = acc.prod * r;
  acc.expo += __builtin_amdgcn_frexp_exp(pr);
  acc.prod = __builtin_amdgcn_frexp_mant(pr);
}
__device__ __forceinline__ double acc_total(const ChainAcc &acc) {
  return acc.logw + log(acc.prod) + (double)acc.expo * 0.69314718055994530942;
}
// c = d / r from the hardware reciprocal estimate refined by two
// Newton-Raphson steps (quadratic convergence to a few ulp of 1/r)
__device__ __forceinline__ double div_nr(double d, double r) {
  double y = __builtin_amdgcn_rcp(r);
  double e = fma(-r, y, 1.0);
  y = fma(y, e, y);
  e = fma(-r, y, 1.0);
  y = fma(y, e, y);
  return d * y;
}

// Row slots of the register tile.  The 2T rows of a lane's tile sit in its
// registers in a lane-dependent order: slot s holds row s ^ key of the
// lane's row group, key depending on the column-group bits (b0, b1, b2) of
// the lane.  With that order the sums of u = M^{-1} x over the eight lanes of
// a column group are taken as a reduce-scatter (row_half_mirror, then the
// quad exchanges xor 1 and xor 2, each step halving the rows a lane carries,
// so that every partner holds in its sent slots the rows the lane keeps) and
// the full vector u comes back by the mirrored all-gather, instead of a full
// butterfly per row.  T = 4: 8 rows, key = (2 b0 + b1) ^ 7 b2; T = 2: 4 rows,
// key = b0 ^ 3 b2 (lanes that differ in b1 share their row).  T = 1 keeps
// the row order and the full butterflies: for two rows per lane the
// reduce-scatter saves no instruction.
template <int T>
__device__ __forceinline__ int tile_key(int bc) {
  const int b0 = bc & 1, b1 = (bc >> 1) & 1, b2 = (bc >> 2) & 1;
  (void)b1;
  if constexpr (T == 4) return (2 * b0 + b1) ^ (b2 ? 7 : 0);
  else if constexpr (T == 2) return b0 ^ (b2 ? 3 : 0);
  else return 0;
}
// u of the lane's 2T row slots from the partial sums t over its T columns,
// and the lane's share of p . u: each row's partial of a = sum_rows p u is
// counted by exactly one lane of the column group
template <int T>
__device__ __forceinline__ double tile_u(double (&t)[2 * T], const double (&pv)[2 * T], int bc, double (&u)[2 * T]) {
  if constexpr (T == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] += dpp_d<0x141>(t[4 + k]);   // row_half_mirror
#pragma unroll
    for (int k = 0; k < 2; ++k) t[k] += dpp_d<0xB1>(t[2 + k]);    // quad_perm [1,0,3,2]
    t[0] += dpp_d<0x4E>(t[1]);                                      // quad_perm [2,3,0,1]
    u[0] = t[0];
    u[1] = dpp_d<0x4E>(u[0]);
    u[2] = dpp_d<0xB1>(u[0]);
    u[3] = dpp_d<0xB1>(u[1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) u[4 + k] = dpp_d<0x141>(u[k]);
    return pv[0] * t[0];
  } else if constexpr (T == 2) {
#pragma unroll
    for (int k = 0; k < 2; ++k) t[k] += dpp_d<0x141>(t[2 + k]);
    t[0] += dpp_d<0xB1>(t[1]);
    t[0] += dpp_d<0x4E>(t[0]);
    u[0] = t[0];
    u[1] = dpp_d<0xB1>(u[0]);
    u[2] = dpp_d<0x141>(u[0]);
    u[3] = dpp_d<0x141>(u[1]);
    return (bc & 2) ? 0.0 : pv[0] * t[0];
  } else {
    static_assert(T == 4 || T == 2, "tile_u serves T = 2 and 4");
    return 0.0;
  }
}
// Column slots likewise: slot c of a lane holds column c ^ ckey of its column
// group, ckey depending on the lowest row-group bit a0 (lane bit 3), so that
// the sums of w = p M^{-1} over the four row groups start with a
// reduce-scatter over a0 (row_ror:8), take the sum over the other row-group
// bit on the half as many values (permlane16 pairs) and end with the
// all-gather over a0.  T = 4: ckey = 2 a0; T = 2: ckey = a0; T = 1: none.
template <int T>
__device__ __forceinline__ int tile_ckey(int ar) {
  if constexpr (T == 4) return 2 * (ar & 1);
  else if constexpr (T == 2) return ar & 1;
  else return 0;
}
// sum of a value over the two 16-lane rows of each 32-lane half, the same
// bits in every lane (the second step of sum_ar)
__device__ __forceinline__ double sum_r16(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
template <int T>
__device__ __forceinline__ void tile_w(double (&t)[T], double (&wv)[T]) {
  if constexpr (T == 4) {
    t[0] += dpp_d<0x128>(t[2]);   // row_ror:8
    t[1] += dpp_d<0x128>(t[3]);
    wv[0] = sum_r16(t[0]);
    wv[1] = sum_r16(t[1]);
    wv[2] = dpp_d<0x128>(wv[0]);
    wv[3] = dpp_d<0x128>(wv[1]);
  } else if constexpr (T == 2) {
    t[0] += dpp_d<0x128>(t[1]);
    wv[0] = sum_r16(t[0]);
    wv[1] = dpp_d<0x128>(wv[0]);
  } else {
    wv[0] = sum_ar(t[0]);
  }
}

// Accepted flips of a chunk are returned as a bit mask (bit r = row r of the
// chunk); the field flip and the row scaling Phi_R[i,:] *= 1 + Delta are
// applied by flush_chunk, since no later site of the slice reads them.
template <int T, typename PE>
__device__ unsigned chain_chunk_reg(const WalkerDesc &w, double (&M)[2 * T][T], const double *xsb_g, int mm,
                                    const PE *prow_g, int ldp, const double *usb_g, const double *dsb_g, int cnt,
                                    int S, ChainAcc &acc) {
  const int lane = TID & 63, sp = lane >> 5, h = lane & 31, ar = h >> 3, bc = h & 7;
  const int m = w.ne[sp], key = tile_key<T>(bc), ckey = tile_ckey<T>(ar);
  const lds_f64 *xsp = as_lds(xsb_g) + sp * S * mm + bc * T;
  const lds_f64 *usb = as_lds(usb_g);
  const lds_f64 *dsb = as_lds(dsb_g) + sp * S;
  // right-row columns outside 0..m-1 are read from column 0: the matching
  // rows and columns of the register inverse are zero, so they add nothing
  decltype(as_lds(prow_g)) prow[2 * T];
#pragma unroll
  for (int i = 0; i < 2 * T; ++i) {
    const int a = ar * 2 * T + (i ^ key);
    prow[i] = as_lds(prow_g) + (a < m ? a : 0);
  }
  struct Row {
    double x[T], p[2 * T], u, d;
  };
  auto load = [&](int r, Row &R) {
#pragma unroll
    for (int j = 0; j < T; ++j) R.x[j] = xsp[r * mm + (j ^ ckey)];
#pragma unroll
    for (int i = 0; i < 2 * T; ++i) R.p[i] = (double)prow[i][r * ldp];
    R.d = dsb[r];
    R.u = usb[r];
  };
  unsigned mask = 0;
  auto step = [&](int r, const Row &R) {
    const double delta = R.d;
    double u[2 * T], t[2 * T];
#pragma unroll
    for (int i = 0; i < 2 * T; ++i) {
      t[i] = M[i][0] * R.x[0];
#pragma unroll
      for (int j = 1; j < T; ++j) t[i] = fma(M[i][j], R.x[j], t[i]);
    }
    double wv[T], tw[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      tw[j] = R.p[0] * M[0][j];
#pragma unroll
      for (int i = 1; i < 2 * T; ++i) tw[j] = fma(R.p[i], M[i][j], tw[j]);
    }
    tile_w<T>(tw, wv);
    double a;
    if constexpr (T == 1) {
      double ap = 0.0;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        u[i] = sum_bc(t[i]);
        ap = fma(R.p[i], u[i], ap);
      }
      a = sum_ar(ap);
    } else {
      // u for the update; a = (p M^{-1}) . x over the lane's columns, then
      // over the column groups (w is the same in the four row groups)
      tile_u<T>(t, R.p, bc, u);
      double xa = wv[0] * R.x[0];
#pragma unroll
      for (int j = 1; j < T; ++j) xa = fma(wv[j], R.x[j], xa);
      a = sum_bc(xa);
    }
    const double rsp = fma(delta, a, 1.0);
    const double ratio = halves_product(rsp);
    acc.nnear += near_tie(R.u, fabs(ratio));
    // ratio and the uniform are identical in every lane: a scalar branch
    if (accept_site(R.u, fabs(ratio))) {
      const double c = div_nr(delta, rsp);
      if constexpr (T == 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double cu = c * u[i];
          M[i][0] = fma(-cu, wv[0], M[i][0]);
        }
      } else {
        double cw[T];
#pragma unroll
        for (int j = 0; j < T; ++j) cw[j] = c * wv[j];
#pragma unroll
        for (int i = 0; i < 2 * T; ++i)
#pragma unroll
          for (int j = 0; j < T; ++j) M[i][j] = fma(-u[i], cw[j], M[i][j]);
      }
      mask |= 1u << r;
      acc_ratio(acc, fabs(ratio));
    }
  };
  // loads are issued one site ahead and unconditionally (a row past the end
  // of the chunk is read again from its last row) so that waits can count
  // exactly the loads still in flight
  Row R0, R1;
  const int last = cnt - 1;
  if (cnt > 0) load(0, R0);
  for (int r = 0; r < cnt; r += 2) {
    load(min(r + 1, last), R1);
    step(r, R0);
    if (r + 1 >= cnt) break;
    load(min(r + 2, last), R0);
    step(r + 1, R1);
  }
  acc.nacc += __builtin_popcount(mask);
  return mask;
}

// Version with the inverse in memory (LDS for Ne <= 64, the walker's device
// scratch above), for any Ne.  The inverse M (row-major) is kept together
// with a column-major copy MT for the block, so that every lane walks
// consecutive addresses: lane h of a half owns rows and columns h, h + 32, ...
// of its spin's inverse, forms u_h = M[h,:] x from MT and w_h = p M[:,h]
// from M, and takes the rank-1 update of column h of M and of column h of MT
// (row h of M) with the same fused products, so the two stay exact transposes.
// sum_b A[b * sa] x[b] over b < m in blocks of 8 (eight loads in flight,
// eight independent accumulators)
template <typename PA, typename PX>
__device__ __forceinline__ double dot8(PA A, int sa, PX x, int m) {
  double t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) t[e] = 0.0;
  int b = 0;
  for (; b + 8 <= m; b += 8) {
    double av[8], xv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = A[(b + e) * sa];
      xv[e] = (double)x[b + e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = fma(av[e], xv[e], t[e]);
  }
  for (; b < m; ++b) t[0] = fma(A[b * sa], (double)x[b], t[0]);
  return ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
}
// A[b * sa] = fma(-k_b, v_b, A[b * sa]) for b < m in blocks of 8, with
// k_b = kc * kv[b] (kc alone when kv is null) and v_b = v[b] (vc when v is null)
__device__ __forceinline__ void axpy8(double *A, int sa, double kc, const double *kv, const double *v, double vc,
                                      int m) {
  int b = 0;
  for (; b + 8 <= m; b += 8) {
    double av[8], vv[8], kk[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = A[(b + e) * sa];
      vv[e] = v ? v[b + e] : vc;
      kk[e] = kv ? kc * kv[b + e] : kc;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) A[(b + e) * sa] = fma(-kk[e], vv[e], av[e]);
  }
  for (; b < m; ++b) A[b * sa] = fma(-(kv ? kc * kv[b] : kc), v ? v[b] : vc, A[b * sa]);
}

// Version with the inverse in memory (LDS for Ne <= 64, the walker's device
// scratch above), for any Ne.  The inverse M (row-major) is kept together
// with a column-major copy MT for the block, so that every lane walks
// consecutive addresses: lane h of a half owns rows and columns h, h + 32, ...
// of its spin's inverse, forms u_h = M[h,:] x from MT and w_h = p M[:,h]
// from M, and takes the rank-1 update of column h of M and of column h of MT
// (row h of M) with the same fused products, so the two stay exact transposes.
template <typename PE>
__device__ unsigned chain_chunk_lds(const WalkerDesc &w, Lds &L, const double *xsb, int mm, const PE *prow,
                                    int ldp, const double *usb, const int8_t *fsb, int cnt, int S, ChainAcc &acc) {
  const int lane = TID & 63, sp = lane >> 5, h = lane & 31;
  const int m = w.ne[sp];
  double *M = sp ? L.Ms1 : L.Ms0;
  double *MT = sp ? L.B : L.A;
  double *ush = L.uw + sp * 2 * L.vs;   // u of the current site, then w on acceptance
  double *wsh = ush + L.vs;
  const double *xsp = xsb + sp * S * mm;
  unsigned mask = 0;
  for (int r = 0; r < cnt; ++r) {
    const double *xrow = xsp + r * mm;
    const PE *pr = prow + r * ldp;
    const int sv = fsb[r];
    const int ss = sp == 0 ? sv : -sv;
    const double delta = ss > 0 ? w.delta_dn_s : w.delta_up_s;
    double part = 0.0;
#pragma unroll 1
    for (int row = h; row < m; row += 32) {
      const double u = dot8(MT + row, m, xrow, m);
      ush[row] = u;
      part = fma((double)pr[row], u, part);
    }
    for (int o = 16; o >= 1; o >>= 1) part += __shfl_xor(part, o);
    const double rsp = 1.0 + delta * part;
    const double ratio = lane_read(rsp, 0) * lane_read(rsp, 32);
    acc.nnear += near_tie(usb[r], fabs(ratio));
    if (accept_site(usb[r], fabs(ratio))) {
#pragma unroll 1
      for (int col = h; col < m; col += 32) wsh[col] = dot8(M + col, m, pr, m);
      wave_fence();
      const double c = delta / rsp;
      // element (a, b) of M and (b, a) of MT both take fma(-(c u_a), w_b, .)
#pragma unroll 1
      for (int h2 = h; h2 < m; h2 += 32) {
        axpy8(MT + h2, m, c * ush[h2], nullptr, wsh, 0.0, m);
        axpy8(M + h2, m, c, ush, nullptr, wsh[h2], m);
      }
      mask |= 1u << r;
      acc_ratio(acc, fabs(ratio));
      acc.nacc += 1;
      wave_fence();
    }
  }
  return mask;
}

// ---------------------------------------------------------------------------
// Delayed (submatrix) flip chain, for any Ne.  Per staged chunk of cnt sites
// and per spin, with x_r the left rows, p_r the right rows and M = M^{-1}:
//   U = M X (Ne x cnt),  W = P M (cnt x Ne),  G = P U (cnt x cnt)
// (all waves).  Wave 0 then decides the sites in order on G alone: site r
// has a_r = G[r][r], and an accepted site moves the rest of the chunk by
// G <- G - c_r G[:, r] G[r, :] (the Sherman-Morrison term seen through P and
// X).  Finally (all waves) the inverse takes the k accepted terms at once:
//   u~_t = U[:, r_t] - sum_{t'<t} c_t' G_t'[r_t', r_t] u~_t',
//   w~_t = W[r_t, :] - sum_{t'<t} c_t' G_t'[r_t, r_t'] w~_t',
//   M <- M - sum_t c_t u~_t w~_t^T,
// which is the sequence of rank-1 updates of the site-by-site chain with M
// read three times per chunk instead of per site.  G_t' is G when site r_t'
// was accepted; its row and column r_t' are recorded then.
// ---------------------------------------------------------------------------
struct DelayedBufs {
  double *U, *W, *Ut, *Wt, *rrec, *crec;
};
__device__ __forceinline__ DelayedBufs dbufs(const WalkerDesc &w, int sp) {
  const size_t mb = (size_t)w.mmax * kDS;
  double *base = w.dch + (size_t)sp * 4 * mb;
  double *rec = w.dch + 8 * mb;
  return DelayedBufs{base, base + mb, base + 2 * mb, base + 3 * mb, rec + (size_t)sp * kDS * kDS,
                     rec + (size_t)(2 + sp) * kDS * kDS};
}

// U, W, then G into LDS (all threads); ends with a barrier.  KS >= cnt.
// A thread takes one row a of U (all sites at once: each block of eight
// entries of M row a serves every site) or one column b of W (likewise with
// M column b, read side by side across threads).
template <int KS, typename PE>
__device__ __forceinline__ void delayed_prologue(const WalkerDesc &w, Lds &L, const double *xsb, int xld, const PE *const prow[2],
                                 const int ldp[2], int cnt, int S) {
  const int m0 = w.ne[0], m1 = w.ne[1];
  for (int e = TID; e < 2 * (m0 + m1); e += kThreads) {
    const bool isw = e >= m0 + m1;
    const int f = isw ? e - (m0 + m1) : e;
    const int sp = f < m0 ? 0 : 1, idx = f < m0 ? f : f - m0, m = sp ? m1 : m0;
    const double *M = sp ? L.Ms1 : L.Ms0;
    const DelayedBufs B = dbufs(w, sp);
    double acc[KS];
#pragma unroll
    for (int r = 0; r < KS; ++r) acc[r] = 0.0;
    if (!isw) {
      // U[a][r] = sum_b M[a][b] X[r][b]
      const double *Mr = M + (size_t)idx * m;
      const double *X = xsb + (size_t)sp * S * xld;
      int b0 = 0;
      double mn[8];
      if (m >= 8)
#pragma unroll
        for (int q = 0; q < 8; ++q) mn[q] = Mr[q];
      for (; b0 + 8 <= m; b0 += 8) {
        double mv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) mv[q] = mn[q];
        if (b0 + 16 <= m)   // the next block's loads go out before this block's arithmetic
#pragma unroll
          for (int q = 0; q < 8; ++q) mn[q] = Mr[b0 + 8 + q];
#pragma unroll
        for (int r = 0; r < KS; ++r)
          if (r < cnt)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[r] = fma(mv[q], X[r * xld + b0 + q], acc[r]);
      }
      for (; b0 < m; ++b0) {
        const double mv = Mr[b0];
#pragma unroll
        for (int r = 0; r < KS; ++r)
          if (r < cnt) acc[r] = fma(mv, X[r * xld + b0], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < KS; ++r)
        if (r < cnt) B.U[idx * kDS + r] = acc[r];
    } else {
      // W[r][b] = sum_a P[r][a] M[a][b]
      const PE *P = prow[sp];
      const int lp = ldp[sp];
      int a0 = 0;
      double mn[8];
      if (m >= 8)
#pragma unroll
        for (int q = 0; q < 8; ++q) mn[q] = M[(size_t)q * m + idx];
      for (; a0 + 8 <= m; a0 += 8) {
        double mv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) mv[q] = mn[q];
        if (a0 + 16 <= m)
#pragma unroll
          for (int q = 0; q < 8; ++q) mn[q] = M[(size_t)(a0 + 8 + q) * m + idx];
#pragma unroll
        for (int r = 0; r < KS; ++r)
          if (r < cnt)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[r] = fma((double)P[r * lp + a0 + q], mv[q], acc[r]);
      }
      for (; a0 < m; ++a0) {
        const double mv = M[(size_t)a0 * m + idx];
#pragma unroll
        for (int r = 0; r < KS; ++r)
          if (r < cnt) acc[r] = fma((double)P[r * lp + a0], mv, acc[r]);
      }
#pragma unroll
      for (int r = 0; r < KS; ++r)
        if (r < cnt) B.W[r * w.mmax + idx] = acc[r];
    }
  }
  SYNC();
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    const PE *P = prow[sp];
    const int lp = ldp[sp];
    const DelayedBufs B = dbufs(w, sp);
    double *G = L.dg + sp * kDS * kDS;
    for (int e = TID; e < cnt * cnt; e += kThreads) {
      const int r = e / cnt, s2 = e - r * cnt;
      G[r * kDS + s2] = dot8(B.U + s2, kDS, P + r * lp, m);
    }
  }
  SYNC();
}

// The sequential decisions on G (wave 0; lanes 0..31 spin up, 32..63 spin
// down, lane j holding column j of its spin's G).  Records c_t and the
// accepted sites for the epilogue; returns the accepted-site mask.
__device__ __forceinline__ unsigned delayed_chain(const WalkerDesc &w, Lds &L, const double *usb_g, const double *dsb_g, int cnt,
                                  int S, ChainAcc &acc) {
  const int lane = TID & 63, sp = lane >> 5, j = lane & 31;
  lds_f64 *G = as_lds(L.dg) + sp * kDS * kDS;
  const lds_f64 *usb = as_lds(usb_g);
  const lds_f64 *dsb = as_lds(dsb_g) + sp * S;
  const DelayedBufs B = dbufs(w, sp);
  double *cacc = L.vec + sp * kDS;
  int *accr = L.iscal + 64;
  unsigned mask = 0;
  int k = 0;
  for (int r = 0; r < cnt; ++r) {
    const double delta = dsb[r];
    const double rsp = fma(delta, (double)G[r * kDS + r], 1.0);
    const double ratio = halves_product(rsp);
    acc.nnear += near_tie(usb[r], fabs(ratio));
    // ratio and the uniform are identical in every lane: a scalar decision
    if (accept_site(usb[r], fabs(ratio))) {
      const double c = div_nr(delta, rsp);
      if (j < cnt) {
        const double grow = G[r * kDS + j], gcol = G[j * kDS + r];
        B.rrec[k * kDS + j] = grow;
        B.crec[k * kDS + j] = gcol;
        if (j > r) {
          const double cg = c * grow;
          for (int i = r + 1; i < cnt; ++i) G[i * kDS + j] = fma(-cg, (double)G[i * kDS + r], (double)G[i * kDS + j]);
        }
      }
      if (j == 0) cacc[k] = c;
      if (lane == 0) accr[k] = r;
      ++k;
      mask |= 1u << r;
      acc_ratio(acc, fabs(ratio));
      wave_fence();
    }
  }
  if (lane == 0) L.iscal[100] = k;
  acc.nacc += k;
  return mask;
}

// u~, w~ and the rank-k update of the inverse (all threads); ends with a
// barrier.  The recursion coefficients c_t' G_t'[r_t', r_t] and
// c_t' G_t'[r_t, r_t'] go to LDS (over the chunk matrix, no longer needed);
// a thread carries one row of u~ (then c_t u~_t[a] goes to cu, the staging
// half of the finished chunk) or one column b of w~ in registers, and the
// thread of column b applies M[:, b] -= sum_t c_t u~_t w~_t[b].  KS >= k.
template <int KS>
__device__ __forceinline__ void delayed_epilogue(const WalkerDesc &w, Lds &L, double *cu, int cu_ld, int cu_sp) {
  const int k = L.iscal[100];
  if (k == 0) return;
  const int *accr = L.iscal + 64;
  double *CU = L.dg, *CW = L.dg + 2 * kDS * kDS;
  for (int e = TID; e < 2 * k * k; e += kThreads) {
    const int sp = e / (k * k), rem = e - sp * k * k, t2 = rem / k, t = rem - t2 * k;
    const DelayedBufs B = dbufs(w, sp);
    const double c2 = L.vec[sp * kDS + t2];
    CU[sp * kDS * kDS + t2 * kDS + t] = c2 * B.rrec[t2 * kDS + accr[t]];
    CW[sp * kDS * kDS + t2 * kDS + t] = c2 * B.crec[t2 * kDS + accr[t]];
  }
  SYNC();
  const int m0 = w.ne[0], m1 = w.ne[1];
  // rows of u~ (c_t u~_t[a] into cu[sp][t][a])
  for (int f = TID; f < m0 + m1; f += kThreads) {
    const int sp = f < m0 ? 0 : 1, a = f < m0 ? f : f - m0;
    const DelayedBufs B = dbufs(w, sp);
    const double *cf = CU + sp * kDS * kDS;
    double v[KS];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      v[t] = 0.0;
      if (t < k) {
        double x = B.U[a * kDS + accr[t]];
#pragma unroll
        for (int t2 = 0; t2 < t; ++t2) x = fma(-cf[t2 * kDS + t], v[t2], x);
        v[t] = x;
        cu[(size_t)sp * cu_sp + t * cu_ld + a] = L.vec[sp * kDS + t] * x;
      }
    }
  }
  SYNC();
  // columns of w~, then the update of column b of M
  for (int f = TID; f < m0 + m1; f += kThreads) {
    const int sp = f < m0 ? 0 : 1, b = f < m0 ? f : f - m0, m = sp ? m1 : m0;
    const DelayedBufs B = dbufs(w, sp);
    const double *cf = CW + sp * kDS * kDS;
    double v[KS];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      v[t] = 0.0;
      if (t < k) {
        double x = B.W[accr[t] * w.mmax + b];
#pragma unroll
        for (int t2 = 0; t2 < t; ++t2) x = fma(-cf[t2 * kDS + t], v[t2], x);
        v[t] = x;
      }
    }
    double *M = sp ? L.Ms1 : L.Ms0;
    const double *cus = cu + (size_t)sp * cu_sp;
    // eight rows at a time: their loads of M are in flight together
    int a = 0;
    for (; a + 8 <= m; a += 8) {
      double mv[8], s2[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        mv[q] = M[(size_t)(a + q) * m + b];
        s2[q] = 0.0;
      }
#pragma unroll
      for (int t = 0; t < KS; ++t)
        if (t < k)
#pragma unroll
          for (int q = 0; q < 8; ++q) s2[q] = fma(cus[t * cu_ld + a + q], v[t], s2[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) M[(size_t)(a + q) * m + b] = mv[q] - s2[q];
    }
    for (; a < m; ++a) {
      double s2 = 0.0;
#pragma unroll
      for (int t = 0; t < KS; ++t)
        if (t < k) s2 = fma(cus[t * cu_ld + a], v[t], s2);
      M[(size_t)a * m + b] -= s2;
    }
  }
  SYNC();
}

// ---------------------------------------------------------------------------
// Delayed flip chain on the FP64 matrix cores (shape kMfma).  Per chunk of
// 16 sites (one 16-wide tile) and per spin, with x_r the left rows, p_r the
// right rows, M = M^{-1} and D = diag(Delta_r):
//   U = M X (Ne x 16),  W = P M (16 x Ne),  G = P U (16 x 16)        [MFMA]
// Wave 0 then decides the sites in order on G alone, by Gauss-Jordan sweeps
// of A = I + G D (both spins, one in each half of the wave): the pivot of
// site r is 1 + Delta_r G_t[r][r], the spin's ratio r_s with every earlier
// accepted site of the chunk applied (a Schur complement), and an accepted
// site is swept.  Once the accepted set S is swept, A[S,S] = -(I + G_SS D_S)^-1,
// so the Woodbury identity gives the inverse of the flipped system,
//   M <- M - U_S D_S (I + G_SS D_S)^{-1} W_S = M - U (Z W),
//   Z = -D A[S,S] (zero outside S),                                   [MFMA]
// the product of the chunk's Sherman-Morrison updates (main text, delay and
// submatrix updates of the auxiliary-field sweep).
// Operand layouts of v_mfma_f64_16x16x4f64 (lane l, c = l % 16, g = l / 16):
// A (16 x 4) holds A[c][g], B (4 x 16) holds B[g][c], and element j of the
// 16 x 16 result holds D[4 j + g][c].
// ---------------------------------------------------------------------------

// The chain's chunk matrices.  U (Ne16 x 17 per spin, for the update) in LDS
// or, when the launch has no room, in the walker's device scratch; the two
// partial G of each spin (16 x 16, in MFMA result order) and G then Z
// (16 x 17) in LDS.  W and Y never leave the registers of the wave that owns
// their column tile.
struct MfBufs {
  double *U[2];
  double *GP[2];   // [2 partials][4 x 64]
  double *GZ[2];
};
__device__ __forceinline__ MfBufs mfbufs(const WalkerDesc &w, double *dg, bool u_lds) {
  MfBufs b;
  b.GZ[0] = dg;
  b.GZ[1] = dg + 16 * 17;
  b.GP[0] = dg + 2 * 16 * 17;
  b.GP[1] = b.GP[0] + 2 * 256;
  double *base = u_lds ? b.GP[1] + 2 * 256 : w.dch;
  b.U[0] = base;
  b.U[1] = base + 17 * ne16(w.ne[0]);
  return b;
}
// U addressed in LDS or device memory
template <typename PU> __device__ __forceinline__ PU uwp(double *p);
template <> __device__ __forceinline__ lds_f64 *uwp<lds_f64 *>(double *p) { return as_lds(p); }
template <> __device__ __forceinline__ double *uwp<double *>(double *p) { return p; }

// Tiles of a chunk: wave w works for spin w / 2; it owns the W (and Y, and
// update) column tiles t with t % 2 == w % 2 and the U row tiles with
// t % 2 != w % 2, so a spin's two waves share its work whatever its tile
// count.  At most kMfTiles column tiles per wave (Ne <= 128).
constexpr int kMfTiles = 4;

// sum_k A[c][k] B[k][.] over k < m for one 16 x 16 result tile, four
// operand groups of four k per round, the next round's loads issued before
// this round's MFMAs; lda(k) and ldb(k) load this lane's operands.
template <typename LA, typename LB>
__device__ __forceinline__ v4d mf_dot(v4d acc, int m, LA &&lda, LB &&ldb) {
  const int g = (TID & 63) >> 4;
  double a[4], b[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + g;
      a[u] = k < m ? lda(k) : 0.0;
      b[u] = k < m ? ldb(k) : 0.0;
    }
  };
  if (m > 0) load(0);
  for (int k0 = 0; k0 < m; k0 += 16) {
    double a0[4], b0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { a0[u] = a[u]; b0[u] = b[u]; }
    if (k0 + 16 < m) load(k0 + 16);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + 4 * u < m) acc = mfma_f64(a0[u], b0[u], acc);
  }
  return acc;
}

// Phase A (all waves): W tiles into registers; U tiles to U (LDS or device
// memory) and, from their registers, the spin's partial G = P U of this
// wave.  PM: the inverses; PP: the right rows (LDS, resident or staged).
template <typename PU, typename PM, typename PP>
__device__ __forceinline__ void mf_front(const WalkerDesc &w, const MfBufs &B, PM M0, PM M1, const double *xsb,
                                         int xld, PP P0, PP P1, int lp0, int lp1, int cnt, v4d (&Wr)[kMfTiles]) {
  const int lane = TID & 63, wave = TID >> 6, c = lane & 15, g = lane >> 4;
  const int sp = wave >> 1, par = wave & 1, m = w.ne[sp], T = ne16(m) >> 4;
  const PM M = sp ? M1 : M0;
  const PP P = sp ? P1 : P0;
  const int lp = sp ? lp1 : lp0;
  const bool cok = c < cnt;
  const lds_f64 *X = as_lds(xsb) + sp * kMS * xld;
  // W[r][16t + i] = sum_k P[r][k] M[k][16t + i]
#pragma unroll
  for (int s = 0; s < kMfTiles; ++s) {
    const int t = 2 * s + par;
    Wr[s] = (v4d){0.0, 0.0, 0.0, 0.0};
    if (t < T) {
      const int col = 16 * t + c;
      const bool colok = col < m;
      Wr[s] = mf_dot(Wr[s], m, [&](int k) { return cok ? (double)P[c * lp + k] : 0.0; },
                     [&](int k) { return colok ? (double)M[k * m + col] : 0.0; });
    }
  }
  // U[16t + i][r] = sum_k M[16t + i][k] X[r][k]; then G += P[:, tile t] U_t
  // with U_t's registers as the B operand (element j holds row 4j + g)
  v4d gp = {0.0, 0.0, 0.0, 0.0};
  PU U = uwp<PU>(B.U[sp]);
  for (int t = 1 - par; t < T; t += 2) {
    const int row = 16 * t + c;
    const bool rok = row < m;
    const v4d ut = mf_dot((v4d){0.0, 0.0, 0.0, 0.0}, m, [&](int k) { return rok ? (double)M[row * m + k] : 0.0; },
                          [&](int k) { return cok ? X[c * xld + k] : 0.0; });
#pragma unroll
    for (int j = 0; j < 4; ++j) U[(16 * t + 4 * j + g) * 17 + c] = ut[j];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 16 * t + 4 * u;
      if (k < m) gp = mfma_f64((cok && k + g < m) ? (double)P[c * lp + k + g] : 0.0, ut[u], gp);
    }
  }
  lds_f64 *G = as_lds(B.GP[sp]) + par * 256;
#pragma unroll
  for (int j = 0; j < 4; ++j) G[j * 64 + lane] = gp[j];
}

// One site of the decision chain (R fixed at compile time: the DPP row
// broadcast takes its source lane as an immediate).  Lane (s, h, j) =
// 32 s + 16 h + j holds rows 8h..8h+7 of column j of spin s's A = I + G D.
struct MfSweep {
  double a[8];
  unsigned mask;
  int nnear;
  double prod;   // accepted-ratio product of the chunk, renormalised as in acc_ratio
  int expo;
};
// a[q] <- a[q] + b * (a[q] of lane R of this lane's 16-lane row) for the
// eight rows, one 64-bit DPP instruction each (row broadcast); the s_nop
// covers a write of a broadcast register by the instruction just before
template <int R>
__device__ __forceinline__ void fma_bcast8(double (&a)[8], double b) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %0, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %1, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %2, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %3, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %4, %4, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %5, %5, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %6, %6, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %7, %7, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
      : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7])
      : "v"(b), "n"(R));
}
template <int R>
__device__ __forceinline__ void mf_site(MfSweep &S, int sp, int h, int j, double uu, int cnt) {
  constexpr int HR = R >> 3, QR = R & 7;
  if (R < cnt) {
    // pivots of both spins (uniform), the ratio and the uniform of site R
    const double pu = lane_read(S.a[QR], 16 * HR + R), pd = lane_read(S.a[QR], 32 + 16 * HR + R);
    const double ratio = pu * pd;
    const double ur = lane_read(uu, R);
    S.nnear += near_tie(ur, fabs(ratio));
    if (accept_site(ur, fabs(ratio))) {
      const double pinv = div_nr(1.0, sp ? pd : pu);
      // row R of this lane's column (held by the half HR)
      const unsigned lo = (unsigned)__double2loint(S.a[QR]), hi = (unsigned)__double2hiint(S.a[QR]);
      const auto xl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
      const auto xh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
      const double rowv = __hiloint2double((int)xh[HR], (int)xl[HR]);
      const bool isr = j == R;
      // A[i][j] -= A[i][R] A[R][j] / p; column R itself: A[i][R] <- A[i][R] / p,
      // i.e. A - A (1 - 1/p); A[i][R] comes from lane R of the 16-lane row
      const double nt = isr ? pinv - 1.0 : -(rowv * pinv);
      const double pr_new = isr ? -pinv : rowv * pinv;
      fma_bcast8<R>(S.a, nt);
      if (h == HR) S.a[QR] = pr_new;
      S.mask |= 1u << R;
      const double pr = S.prod * fabs(ratio);
      S.expo += __builtin_amdgcn_frexp_exp(pr);
      S.prod = __builtin_amdgcn_frexp_mant(pr);
    }
  }
  if constexpr (R + 1 < kMS) mf_site<R + 1>(S, sp, h, j, uu, cnt);
}

// Phase B (wave 0): A = I + G D with G the sum of the spin's two partials,
// Gauss-Jordan sweeps of the accepted sites, then Z = -D A[S,S] into GZ.
// Returns the accepted-site mask.
__device__ __forceinline__ unsigned mf_decide(const MfBufs &B, const double *usb_g, const double *dsb_g, int cnt,
                                              int S, ChainAcc &acc) {
  const int lane = TID & 63, sp = lane >> 5, h = (lane >> 4) & 1, j = lane & 15;
  const lds_f64 *usb = as_lds(usb_g);
  const lds_f64 *dsb = as_lds(dsb_g) + sp * S;
  const lds_f64 *gp = as_lds(B.GP[sp]);
  lds_f64 *gz = as_lds(B.GZ[sp]);
  const double dj = j < cnt ? dsb[j] : 0.0;
  MfSweep st;
  double dr[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int row = 8 * h + q;
    // G[row][j] sits in result element row / 4 of lane 16 (row % 4) + j
    const int ix = (row >> 2) * 64 + (row & 3) * 16 + j;
    st.a[q] = fma(gp[ix] + gp[256 + ix], dj, row == j ? 1.0 : 0.0);
    dr[q] = row < cnt ? dsb[row] : 0.0;
  }
  const double uu = j < cnt ? usb[j] : 2.0;
  st.mask = 0u;
  st.nnear = 0;
  st.prod = 1.0;
  st.expo = 0;
  // the chunk's sites run from registers: the caller's accumulator is
  // folded in once, after the chunk
  mf_site<0>(st, sp, h, j, uu, __builtin_amdgcn_readfirstlane(cnt));
  const unsigned mask = st.mask;
  acc_ratio(acc, st.prod);
  acc.expo += st.expo;
  acc.nnear += st.nnear;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int row = 8 * h + q;
    gz[row * 17 + j] = ((mask >> row) & (mask >> j) & 1u) ? -dr[q] * st.a[q] : 0.0;
  }
  acc.nacc += __builtin_popcount(mask);
  return mask;
}

// Phase C (all waves): for each owned column tile t, Y_t = Z W_t with W_t's
// registers as the B operand, then M[ta, t] -= U[ta, :] Y_t for every row
// tile ta with Y_t's registers as the B operand.
template <typename PU, typename PM>
__device__ __forceinline__ void mf_back(const WalkerDesc &w, const MfBufs &B, PM M0, PM M1,
                                        const v4d (&Wr)[kMfTiles]) {
  const int lane = TID & 63, wave = TID >> 6, c = lane & 15, g = lane >> 4;
  const int sp = wave >> 1, par = wave & 1, m = w.ne[sp], T = ne16(m) >> 4;
  PM M = sp ? M1 : M0;
  const lds_f64 *Z = as_lds(B.GZ[sp]);
  const PU U = uwp<PU>(B.U[sp]);
  double za[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) za[u] = Z[c * 17 + 4 * u + g];
#pragma unroll
  for (int s = 0; s < kMfTiles; ++s) {
    const int t = 2 * s + par;
    if (t >= T) break;
    v4d y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) y = mfma_f64(za[u], Wr[s][u], y);
    const int col = 16 * t + c;
    // the next row tile's operands are loaded before this tile's MFMAs
    v4d cn;
    double an[4];
    auto load = [&](int ta) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * ta + 4 * j + g;
        cn[j] = (row < m && col < m) ? (double)M[row * m + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) an[u] = -(double)U[(16 * ta + c) * 17 + 4 * u + g];
    };
    load(0);
    for (int ta = 0; ta < T; ++ta) {
      v4d acc = cn;
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = an[u];
      if (ta + 1 < T) load(ta + 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma_f64(a[u], y[u], acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * ta + 4 * j + g;
        if (row < m && col < m) M[row * m + col] = acc[j];
      }
    }
  }
}

// One chunk of the matrix-core chain from its staged rows to the updated
// inverse.  Wave 0 decides while waves 1..3 flush the previous chunk and
// stage the next (the caller's callback).  PU: U in LDS or device memory;
// PM: the inverses in LDS or device memory.
template <typename PU, typename PM, typename PP, typename FS>
__device__ __forceinline__ void mf_chunk(const WalkerDesc &w, Lds &L, const MfBufs &B, PM M0, PM M1,
                                         const double *xsb, int xld, PP P0, PP P1, int lp0, int lp1, int cnt,
                                         int bufi, ChainAcc &acc, FS &&side) {
  const int S = L.S;
  v4d Wr[kMfTiles];
  mf_front<PU>(w, B, M0, M1, xsb, xld, P0, P1, lp0, lp1, cnt, Wr);
  SYNC();
  if (TID < 64) {
    const unsigned mask = mf_decide(B, L.us + bufi * S, L.dl + bufi * 2 * S, cnt, S, acc);
    if (TID == 0) L.iscal[8 + bufi] = (int)mask;
  } else {
    side();
  }
  SYNC();
  if (L.iscal[8 + bufi] != 0) {
    mf_back<PU>(w, B, M0, M1, Wr);
    SYNC();
  }
}

// Stage chunk c (rows i0 .. i0+cnt-1) of slice l into buffer bufi: left rows
// (Phi_L'^T = E_K^T Y_l, stored by the left-stack build), right rows when
// streamed, fields and the flip uniforms.  Threads t0.. of the caller.  The
// rows of a chunk are contiguous in device memory; each thread issues eight
// loads (typed as global, so that they are not ordered behind the LDS
// stores) before it stores them into the staging buffer of row stride mm.
typedef __attribute__((address_space(1))) const float gc_f32;
typedef __attribute__((address_space(1))) const double gc_f64;
__device__ __forceinline__ gc_f64 *as_global(const double *p) { return (gc_f64 *)p; }
__device__ __forceinline__ gc_f32 *as_global(const float *p) { return (gc_f32 *)p; }
template <typename F, bool fdiag>
__device__ void stage_chunk_t(const WalkerDesc &w, Lds &L, int l, uint32_t sweep, int i0, int bufi,
                              F *const phi[2], bool resident, int mm, int t0, int nt) {
  if (TID < t0 || TID >= t0 + nt) return;
  const int S = L.S, N = w.N;
  const int cnt = min(S, N - i0);
  const int tid = TID - t0, tot = cnt * mm;
  const int dr = nt / mm, da = nt - dr * mm;
  // every load of the chunk is issued before the first store: the field of
  // this thread's site, then both spins' rows (eight per spin and round)
  const int8_t *srow = w.s + (size_t)(l - 1) * N;
  const int sv = tid < cnt ? (int)srow[i0 + tid] : 0;
  decltype(as_global((const F *)nullptr)) lx[2], pr[2];
  lds_f64 *xd[2], *pd[2];
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    lx[sp] = as_global(reinterpret_cast<const F *>(w.LX[sp]) + ((size_t)(l - 1) * N + i0) * m);
    // (a resident block lives in LDS and is not read here: the global view
    // then points at the left rows, so that no load can leave the buffers)
    pr[sp] = resident ? lx[sp] : as_global((const F *)phi[sp] + (size_t)i0 * m);
    xd[sp] = as_lds(L.xs + (size_t)(bufi * 2 + sp) * S * mm);
    pd[sp] = resident ? nullptr : as_lds(L.ps + (size_t)(bufi * 2 + sp) * S * mm);
  }
  int r = tid / mm, a = tid - r * mm;
  bool first = true;
  for (int e0 = tid; e0 < tot || first; e0 += 8 * nt) {
    double xv[2][8], pv[2][8];
    // D_l of this slice for the streamed right rows (fdiag): the field and
    // onsite factor of each element's row, loaded with the rows and applied
    // at the store, in the storage precision (the product diag_t forms)
    int sr[8];
    double er[8];
    const int r0 = r, a0 = a;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const int m = w.ne[sp];
      r = r0;
      a = a0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = e0 + u * nt < tot && a < m;
        xv[sp][u] = ok ? (double)lx[sp][r * m + a] : 0.0;
        pv[sp][u] = (ok && !resident) ? (double)pr[sp][r * m + a] : 0.0;
        if constexpr (fdiag) {
          if (sp == 0) {
          const int rc = r < cnt ? r : cnt - 1;
          sr[u] = srow[i0 + rc];
          er[u] = w.eps_fac[i0 + rc];
          }
        }
        a += da;
        r += dr;
        if (a >= mm) { a -= mm; ++r; }
      }
    }
    if (first) {
      // the flip uniform and flip factors of this thread's site, while the
      // loads are in flight
      if (tid < cnt) {
        L.us[bufi * S + tid] = uniform01(w.seed, w.wid, kFlip, sweep, (uint32_t)(l - 1), (uint32_t)(i0 + tid));
        L.fs[bufi * S + tid] = (int8_t)sv;
        L.dl[(bufi * 2 + 0) * S + tid] = sv > 0 ? w.delta_dn_s : w.delta_up_s;
        L.dl[(bufi * 2 + 1) * S + tid] = -sv > 0 ? w.delta_dn_s : w.delta_up_s;
      }
      first = false;
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * nt;
        if (e < tot) {
          xd[sp][e] = xv[sp][u];
          if (!resident) {
            if constexpr (fdiag) {
              const int ss = sp == 0 ? sr[u] : -sr[u];
              const F f = (F)((ss > 0 ? w.elam : w.emlam) * er[u]);
              pd[sp][e] = (double)((F)pv[sp][u] * f);
            } else {
              pd[sp][e] = pv[sp][u];
            }
          }
        }
      }
  }
  // sites beyond the threads of the caller (a chunk larger than nt)
  for (int rr = tid + nt; rr < cnt; rr += nt) {
    const int v = srow[i0 + rr];
    L.fs[bufi * S + rr] = (int8_t)v;
    L.us[bufi * S + rr] = uniform01(w.seed, w.wid, kFlip, sweep, (uint32_t)(l - 1), (uint32_t)(i0 + rr));
    L.dl[(bufi * 2 + 0) * S + rr] = v > 0 ? w.delta_dn_s : w.delta_up_s;
    L.dl[(bufi * 2 + 1) * S + rr] = -v > 0 ? w.delta_dn_s : w.delta_up_s;
  }
}

// fdiag is a template argument, and only the chains that may fuse D_l
// (FUSE) carry the fused variant, so that the others keep the staging code
// they had without it
template <bool FUSE, typename F>
__device__ __forceinline__ void stage_d(const WalkerDesc &w, Lds &L, int l, uint32_t sweep, int i0, int bufi,
                                        F *const phi[2], bool resident, int mm, int t0, int nt, bool fdiag) {
  if constexpr (FUSE) {
    if (fdiag) {
      stage_chunk_t<F, true>(w, L, l, sweep, i0, bufi, phi, resident, mm, t0, nt);
      return;
    }
  }
  stage_chunk_t<F, false>(w, L, l, sweep, i0, bufi, phi, resident, mm, t0, nt);
}

// Write back chunk rows after the chain: flip the accepted fields and scale
// the accepted right rows by 1 + Delta (resident rows in place, streamed rows
// on their way back to device memory).  The streamed loop walks the staging
// buffer in the order stage_chunk fills it, so the same thread reads an
// element before it is restaged.
template <typename F>
__device__ void flush_chunk(const WalkerDesc &w, Lds &L, int l, int i0, int bufi, F *const phi[2],
                            bool resident, int mm, int t0, int nt) {
  if (TID < t0 || TID >= t0 + nt) return;
  const int S = L.S, N = w.N;
  const int cnt = min(S, N - i0);
  const unsigned mask = (unsigned)L.iscal[8 + bufi];
  const int8_t *fs = L.fs + bufi * S;
  const int tid = TID - t0;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    auto factor = [&](int r) {
      const int sv = fs[r];
      const int ss = sp == 0 ? sv : -sv;
      return 1.0 + (ss > 0 ? w.delta_dn_s : w.delta_up_s);
    };
    if (resident) {
      if (mask != 0u)
        for (int e = tid; e < cnt * m; e += nt) {
          const int r = e / m, a = e - r * m;
          if ((mask >> r) & 1u) phi[sp][(size_t)(i0 + r) * m + a] *= (F)factor(r);
        }
    } else {
      const lds_f64 *pd = as_lds(L.ps + (size_t)(bufi * 2 + sp) * S * mm);
      F *dst = phi[sp] + (size_t)i0 * m;
      const int tot = cnt * mm, dr = nt / mm, da = nt - dr * mm;
      int r = tid / mm, a = tid - r * mm;
      for (int e = tid; e < tot; e += nt) {
        if (a < m) {
          double v = pd[e];
          if ((mask >> r) & 1u) v *= factor(r);
          dst[r * m + a] = (F)v;
        }
        a += da;
        r += dr;
        if (a >= mm) { a -= mm; ++r; }
      }
    }
  }
  int8_t *srow = w.s + (size_t)(l - 1) * N;
  for (int r = tid; r < cnt; r += nt) {
    const int8_t f = fs[r];
    srow[i0 + r] = ((mask >> r) & 1u) ? (int8_t)(-f) : f;
  }
}

// All slices of block k with the inverse held by wave 0.  On entry D_{l0} has
// been applied and Ms0/Ms1 hold the fresh inverse at the flip point of l0;
// on exit Ms0/Ms1 hold the updated inverse and phi = B_k ... applied.
template <int T, typename F>
__device__ __forceinline__ void forward_block_body(const WalkerDesc &w, int k, uint32_t sweep, Lds &L, F *const phi[2],
                                                   bool resident, int mm, ChainAcc &acc) {
  constexpr bool kReg = T > 0 && T != kDelayed && T != kMfma;   // register-tiled inverse
  // chains that stage D_l with the streamed rows (T = 1 serves Ne <= 8, whose
  // blocks nearly always stay resident, and keeps the staging it had)
  constexpr bool kFuseD = T == 0 || T == 2 || T == 4;
  constexpr int TT = kReg ? T : 1;
  const int N = w.N, S = L.S;
  const int l0 = (k - 1) * w.nstab + 1, l1 = min(k * w.nstab, w.L);
  const int nch = (N + S - 1) / S;
  double M[2 * TT][TT];
  const int lane = TID & 63, sp = lane >> 5, h = lane & 31, ar = h >> 3, bc = h & 7;
  static_assert(T == 0 || T == 1 || T == 2 || T == 4 || T == kDelayed || T == kMfma, "chain shape");
  if constexpr (T == 0) {
    // column-major copies of the inverses for the chain (A, B are free here)
    for (int s2 = 0; s2 < 2; ++s2) {
      const int m = w.ne[s2];
      const double *Ms = s2 ? L.Ms1 : L.Ms0;
      double *MT = s2 ? L.B : L.A;
      for (int t = TID; t < m * m; t += kThreads) {
        const int a = t / m, b = t - (t / m) * m;
        MT[b * m + a] = Ms[t];
      }
    }
    SYNC();
  }
  if constexpr (kReg) {
    if (TID < 64) {
      const int m = w.ne[sp];
      const double *Ms = sp ? L.Ms1 : L.Ms0;
      const int key = tile_key<TT>(bc), ckey = tile_ckey<TT>(ar);
#pragma unroll
      for (int i = 0; i < 2 * T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const int a = ar * 2 * T + (i ^ key), b = bc * T + (j ^ ckey);
          M[i][j] = (a < m && b < m) ? Ms[a * m + b] : 0.0;
        }
    }
  }
  for (int l = l0; l <= l1; ++l) {
    // D_l: applied while a streamed block is staged for the site-by-site
    // chains of kFuseD, whose staging runs beside a longer chain; by a pass
    // for the delayed chains (their staging is the longer side of a chunk,
    // and the fused factors measured slower there than the pass), for
    // resident blocks, and before the block's first slice, where the fresh
    // inverse needs it
    const bool fd = kFuseD && l > l0 && !resident && !(w.flags & 2);
    if (l > l0 && !fd)
      for (int s2 = 0; s2 < 2; ++s2) apply_diag(w, phi[s2], w.ne[s2], l, s2, false);
    if constexpr (T == kDelayed) {
      if (!(w.flags & 2)) {
        stage_d<kFuseD>(w, L, l, sweep, 0, 0, phi, resident, mm, 0, kThreads, fd);
        SYNC();
        for (int c = 0; c < nch; ++c) {
          const int bufi = c & 1, i0 = c * S;
          const int cnt = min(S, N - i0);
          const double *xsb = L.xs + (size_t)bufi * 2 * S * mm;
          auto prologue = [&](auto ks) {
            constexpr int KS = decltype(ks)::value;
            if (resident) {
              const F *pr[2] = {phi[0] + (size_t)i0 * w.ne[0], phi[1] + (size_t)i0 * w.ne[1]};
              const int lp[2] = {w.ne[0], w.ne[1]};
              delayed_prologue<KS>(w, L, xsb, mm, pr, lp, cnt, S);
            } else {
              const double *pr[2] = {L.ps + (size_t)(bufi * 2) * S * mm, L.ps + (size_t)(bufi * 2 + 1) * S * mm};
              const int lp[2] = {mm, mm};
              delayed_prologue<KS>(w, L, xsb, mm, pr, lp, cnt, S);
            }
          };
          if (S <= 8) prologue(std::integral_constant<int, 8>());
          else prologue(std::integral_constant<int, 16>());
          if (TID < 64) {
            const unsigned mask = delayed_chain(w, L, L.us + bufi * S, L.dl + bufi * 2 * S, cnt, S, acc);
            if (TID == 0) L.iscal[8 + bufi] = (int)mask;
          } else {
            if (c >= 1) flush_chunk(w, L, l, (c - 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64);
            if (c + 1 < nch) stage_d<kFuseD>(w, L, l, sweep, (c + 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64, fd);
          }
          SYNC();
          // c u~ goes to this chunk's staging half, free once its rows are consumed
          double *cu = L.xs + (size_t)bufi * 2 * S * mm;
          if (S <= 8) delayed_epilogue<8>(w, L, cu, mm, S * mm);
          else delayed_epilogue<16>(w, L, cu, mm, S * mm);
        }
        flush_chunk(w, L, l, (nch - 1) * S, (nch - 1) & 1, phi, resident, mm, 0, kThreads);
        SYNC();
      }
    } else if constexpr (T == kMfma) {
      if (!(w.flags & 2)) {
        const bool uw_lds = L.dgn >= mfma_lds_doubles(w.ne[0], w.ne[1]);
        const MfBufs mb = mfbufs(w, L.dg, uw_lds);
        const bool mlds = in_lds(L.Ms0);
        stage_d<kFuseD>(w, L, l, sweep, 0, 0, phi, resident, mm, 0, kThreads, fd);
        SYNC();
        for (int c = 0; c < nch; ++c) {
          const int bufi = c & 1, i0 = c * S;
          const int cnt = min(S, N - i0);
          const double *xsb = L.xs + (size_t)bufi * 2 * S * mm;
          auto side = [&]() {
            if (c >= 1) flush_chunk(w, L, l, (c - 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64);
            if (c + 1 < nch) stage_d<kFuseD>(w, L, l, sweep, (c + 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64, fd);
          };
          // right rows from the resident block (storage F, row stride Ne) or
          // the FP64 staging buffer (row stride mm); U, W and the inverses
          // in LDS or device memory
          auto run = [&](auto P0, auto P1, int lp0, int lp1) {
            if (uw_lds) {
              if (mlds) mf_chunk<lds_f64 *>(w, L, mb, as_lds(L.Ms0), as_lds(L.Ms1), xsb, mm, P0, P1, lp0, lp1, cnt, bufi, acc, side);
              else mf_chunk<lds_f64 *>(w, L, mb, L.Ms0, L.Ms1, xsb, mm, P0, P1, lp0, lp1, cnt, bufi, acc, side);
            } else {
              if (mlds) mf_chunk<double *>(w, L, mb, as_lds(L.Ms0), as_lds(L.Ms1), xsb, mm, P0, P1, lp0, lp1, cnt, bufi, acc, side);
              else mf_chunk<double *>(w, L, mb, L.Ms0, L.Ms1, xsb, mm, P0, P1, lp0, lp1, cnt, bufi, acc, side);
            }
          };
          if (resident)
            run(as_lds((const F *)(phi[0] + (size_t)i0 * w.ne[0])), as_lds((const F *)(phi[1] + (size_t)i0 * w.ne[1])),
                w.ne[0], w.ne[1]);
          else
            run(as_lds((const double *)(L.ps + (size_t)(bufi * 2) * S * mm)),
                as_lds((const double *)(L.ps + (size_t)(bufi * 2 + 1) * S * mm)), mm, mm);
        }
        flush_chunk(w, L, l, (nch - 1) * S, (nch - 1) & 1, phi, resident, mm, 0, kThreads);
        SYNC();
      }
    } else if (!(w.flags & 2)) {
      stage_d<kFuseD>(w, L, l, sweep, 0, 0, phi, resident, mm, 0, kThreads, fd);
      SYNC();
      for (int c = 0; c < nch; ++c) {
        const int bufi = c & 1, i0 = c * S;
        const int cnt = min(S, N - i0);
        if (TID < 64) {
          const double *xsb = L.xs + (size_t)bufi * 2 * S * mm;
          const double *us = L.us + bufi * S;
          unsigned mask;
          // right rows: the resident block (storage F) or the FP64 staging buffer
          if (resident) {
            const F *prow = phi[sp] + (size_t)i0 * w.ne[sp];
            const int ldp = w.ne[sp];
            if constexpr (T > 0)
              mask = chain_chunk_reg<T>(w, M, xsb, mm, prow, ldp, us, L.dl + bufi * 2 * S, cnt, S, acc);
            else
              mask = chain_chunk_lds(w, L, xsb, mm, prow, ldp, us, L.fs + bufi * S, cnt, S, acc);
          } else {
            const double *prow = L.ps + (size_t)(bufi * 2 + sp) * S * mm;
            if constexpr (T > 0)
              mask = chain_chunk_reg<T>(w, M, xsb, mm, prow, mm, us, L.dl + bufi * 2 * S, cnt, S, acc);
            else
              mask = chain_chunk_lds(w, L, xsb, mm, prow, mm, us, L.fs + bufi * S, cnt, S, acc);
          }
          if (TID == 0) L.iscal[8 + bufi] = (int)mask;
        } else {
          if (c >= 1) flush_chunk(w, L, l, (c - 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64);
          if (c + 1 < nch) stage_d<kFuseD>(w, L, l, sweep, (c + 1) * S, bufi ^ 1, phi, resident, mm, 64, kThreads - 64, fd);
        }
        SYNC();
      }
      flush_chunk(w, L, l, (nch - 1) * S, (nch - 1) & 1, phi, resident, mm, 0, kThreads);
      SYNC();
    }
    for (int s2 = 0; s2 < 2; ++s2) apply_ek(w, L, phi[s2], w.ne[s2]);
  }
  if constexpr (kReg) {
    if (TID < 64) {
      const int m = w.ne[sp];
      double *Ms = sp ? L.Ms1 : L.Ms0;
      const int key = tile_key<TT>(bc), ckey = tile_ckey<TT>(ar);
#pragma unroll
      for (int i = 0; i < 2 * T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const int a = ar * 2 * T + (i ^ key), b = bc * T + (j ^ ckey);
          if (a < m && b < m) Ms[a * m + b] = M[i][j];
        }
    }
  }
  SYNC();
}
template <int T, typename F>
__device__ void forward_block(const WalkerDesc &w, int k, uint32_t sweep, Lds &L, F *const phi[2], bool resident,
                              int mm, ChainAcc &acc) {
  forward_block_body<T, F>(w, k, sweep, L, phi, resident, mm, acc);
}

// ---------------------------------------------------------------------------
// Equal-time estimators (Wick) from A_s = Phi_R M_s^{-1} Phi_L at a fresh
// boundary, accumulated sign-weighted in the observable layout of the ABI.
// q = 0 sums use traces of Ne x Ne sublattice blocks, O(N Ne^2).
// ---------------------------------------------------------------------------
// Scratch per call: T[2] (N x Ne each), Ad[2] (N each), Afull (2 N^2 when N <= 64).
struct MeasScratch {
  double *T[2];
  double *Ad[2];
  double *Afull;
};
__device__ void measure_point(const WalkerDesc &w, double *const PR[2], double *const XL[2], const double *Ms[2],
                              int sgn, Lds &L, double *obs, const MeasScratch &ms) {
  const int N = w.N, ns = w.nsub;
  const double sg = (double)sgn;
  // T_s = Phi_R M_s^{-1}
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    const int tot = N * m;
    for (int t = TID; t < tot; t += kThreads) {
      const int i = t / m, b = t - (t / m) * m;
      double s = 0.0;
      for (int a = 0; a < m; ++a) s += PR[sp][(size_t)i * m + a] * Ms[sp][a * m + b];
      ms.T[sp][t] = s;
    }
  }
  SYNC();
  // diagonal sums: A_ii per spin into T-adjacent scratch (Aw), then reductions
  double docc = 0.0, eon = 0.0, dens = 0.0;
  for (int i = TID; i < N; i += kThreads) {
    double ad[2];
    for (int sp = 0; sp < 2; ++sp) {
      const int m = w.ne[sp];
      double s = 0.0;
      for (int b = 0; b < m; ++b) s += ms.T[sp][(size_t)i * m + b] * XL[sp][(size_t)i * m + b];
      ad[sp] = s;
      ms.Ad[sp][i] = s;
    }
    docc += ad[0] * ad[1];
    eon += w.eps[i] * (ad[0] + ad[1]);
    dens += ad[0] + ad[1];
  }
  docc = wg_sum(docc, L.red);
  eon = wg_sum(eon, L.red);
  dens = wg_sum(dens, L.red);
  // per-sublattice densities n_a^sigma (kept in LDS scalars 32..47)
  for (int a = 0; a < ns; ++a)
    for (int sp = 0; sp < 2; ++sp) {
      double v = 0.0;
      for (int i = TID; i < N; i += kThreads)
        if (w.sub[i] == a) v += ms.Ad[sp][i];
      v = wg_sum(v, L.red);
      if (TID == 0) L.scal[32 + 2 * a + sp] = v;
    }
  SYNC();
  // kinetic term: sum_b h_b (A_ij + A_ji) for both spins
  double ek = 0.0;
  for (int b = TID; b < w.nbonds; b += kThreads) {
    const int i = w.bi[b], j = w.bj[b];
    double s = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
      const int m = w.ne[sp];
      for (int q = 0; q < m; ++q)
        s += ms.T[sp][(size_t)i * m + q] * XL[sp][(size_t)j * m + q] +
             ms.T[sp][(size_t)j * m + q] * XL[sp][(size_t)i * m + q];
    }
    ek += w.bh[b] * s;
  }
  ek = wg_sum(ek, L.red);
  // sublattice traces
  double *szz = obs + 8, *spar = obs + 8 + ns * ns;
  double szz_tot = 0.0, spar_tot = 0.0;
  const int mu = w.ne[0], md = w.ne[1];
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) {
      double same[2];
      for (int sp = 0; sp < 2; ++sp) {
        const int m = w.ne[sp];
        // Y_a = sum_{i in a} X_i^T T_i  (m x m), trace(Y_a Y_b)
        gram(XL[sp], m, ms.T[sp], m, N, L.A, L.red, w.sub, a);
        gram(XL[sp], m, ms.T[sp], m, N, L.B, L.red, w.sub, b);
        double tr = 0.0;
        for (int t = TID; t < m * m; t += kThreads) {
          const int p = t / m, q = t % m;
          tr += L.A[p * m + q] * L.B[q * m + p];
        }
        tr = wg_sum(tr, L.red);
        const double na = L.scal[32 + 2 * a + sp], nb = L.scal[32 + 2 * b + sp];
        same[sp] = na * nb + (a == b ? na : 0.0) - tr;
      }
      const double nua = L.scal[32 + 2 * a], nda = L.scal[33 + 2 * a];
      const double nub = L.scal[32 + 2 * b], ndb = L.scal[33 + 2 * b];
      const double cross = nua * ndb + nda * nub;
      const double zz = 0.25 * (same[0] + same[1] - cross);
      // Z^a = sum_{i in a} X_up,i^T T_dn,i ; Z'^b = sum_{j in b} T_up,j^T X_dn,j
      gram(XL[0], mu, ms.T[1], md, N, L.A, L.red, w.sub, a);
      gram(ms.T[0], mu, XL[1], md, N, L.B, L.red, w.sub, b);
      double d1 = 0.0;
      for (int t = TID; t < mu * md; t += kThreads) d1 += L.A[t] * L.B[t];
      d1 = wg_sum(d1, L.red);
      // Z'^a and Z^b
      gram(ms.T[0], mu, XL[1], md, N, L.A, L.red, w.sub, a);
      gram(XL[0], mu, ms.T[1], md, N, L.B, L.red, w.sub, b);
      double d2 = 0.0;
      for (int t = TID; t < mu * md; t += kThreads) d2 += L.A[t] * L.B[t];
      d2 = wg_sum(d2, L.red);
      const double pm = (a == b ? nua : 0.0) - d1;
      const double mp = (a == b ? nda : 0.0) - d2;
      const double xy = 0.5 * (pm + mp);
      if (TID == 0) {
        szz[a * ns + b] += sg * zz / w.ncells;
        spar[a * ns + b] += sg * xy / w.ncells;
      }
      szz_tot += zz;
      spar_tot += xy;
    }
  if (TID == 0) {
    obs[0] += sg;
    obs[1] += 1.0;
    obs[2] += sg * docc / N;
    obs[3] += sg * ek / N;
    obs[4] += sg * spar_tot / w.ncells;
    obs[5] += sg * szz_tot / w.ncells;
    obs[6] += sg * eon / N;
    obs[7] += sg * dens / N;
  }
  SYNC();
  if (N <= 64) {
    // all-pair correlations from explicit A matrices (small lattices)
    double *Au = ms.Afull, *Ad = ms.Afull + N * N;
    for (int t = TID; t < N * N; t += kThreads) {
      const int i = t / N, j = t % N;
      double su = 0.0, sd = 0.0;
      for (int q = 0; q < mu; ++q) su += ms.T[0][(size_t)i * mu + q] * XL[0][(size_t)j * mu + q];
      for (int q = 0; q < md; ++q) sd += ms.T[1][(size_t)i * md + q] * XL[1][(size_t)j * md + q];
      Au[t] = su;
      Ad[t] = sd;
    }
    SYNC();
    double *ss = obs + 8 + 2 * ns * ns, *nn = ss + N * N, *nu = nn + N * N, *nd = nu + N;
    for (int t = TID; t < N * N; t += kThreads) {
      const int i = t / N, j = t % N;
      const double d = (i == j) ? 1.0 : 0.0;
      const double uu = Au[i * N + i] * Au[j * N + j] + Au[j * N + i] * (d - Au[i * N + j]);
      const double dd = Ad[i * N + i] * Ad[j * N + j] + Ad[j * N + i] * (d - Ad[i * N + j]);
      const double ud = Au[i * N + i] * Ad[j * N + j];
      const double du = Ad[i * N + i] * Au[j * N + j];
      const double zz = 0.25 * (uu + dd - ud - du);
      const double pm = Au[j * N + i] * (d - Ad[i * N + j]);
      const double mp = Ad[j * N + i] * (d - Au[i * N + j]);
      ss[t] += sg * (zz + 0.5 * (pm + mp));
      nn[t] += sg * (uu + dd + ud + du);
    }
    for (int i = TID; i < N; i += kThreads) {
      nu[i] += sg * Au[i * N + i];
      nd[i] += sg * Ad[i * N + i];
    }
    SYNC();
  }
}

// ---------------------------------------------------------------------------
// Right chain from P with a QR at every block end; (Q_k, V_k) stored.
// Returns sum_k sum_j log V_k,jj for spin sp.
// ---------------------------------------------------------------------------
__device__ double right_stack(const WalkerDesc &w, int sp, Lds &L, double *Phi) {
  const int m = w.ne[sp], N = w.N;
  fill_P(w, sp, Phi);
  double ld = 0.0;
  for (int k = 1; k <= w.nblk; ++k) {
    const int l0 = (k - 1) * w.nstab + 1, l1 = min(k * w.nstab, w.L);
    for (int l = l0; l <= l1; ++l) {
      apply_diag(w, Phi, m, l, sp, false);
      apply_ek(w, L, Phi, m);
    }
    double *Q = w.RQ[sp] + (size_t)(k - 1) * N * m;
    double *V = w.RV[sp] + (size_t)(k - 1) * m * m;
    ld += cholqr(Phi, w.T[sp], Q, Phi, V, w.fVp, N, m, L, w.sc);
  }
  return ld;
}

// M = P^T Q_n and its inverse into Minv (global); returns log|det M|, sign.
__device__ __noinline__ void inverse_at_beta(const WalkerDesc &w, int sp, Lds &L, double *logabs, int *sign) {
  const int m = w.ne[sp], N = w.N;
  const double *Qn = w.RQ[sp] + (size_t)(w.nblk - 1) * N * m;
  for (int t = TID; t < m * m; t += kThreads) {
    const int a = t / m, b = t % m;
    L.A[t] = Qn[(size_t)w.occ[sp][a] * m + b];
  }
  SYNC();
  if (m == 0) { *logabs = 0.0; *sign = 1; SYNC(); return; }
  if (!gj_inverse(L.A, w.Minv[sp], m, L, logabs, sign)) {
    if (TID == 0) w.sc->status |= 4;
  }
  SYNC();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_init(const WalkerDesc *__restrict__ descs, int draw_fields, int draw_occ) {
  const WalkerDesc &w = descs[blockIdx.x];
  if (draw_fields) {
    const int tot = w.L * w.N;
    for (int t = TID; t < tot; t += kThreads) {
      const int l = t / w.N, i = t % w.N;
      w.s[t] = uniform01(w.seed, w.wid, kInitField, 0, (uint32_t)l, (uint32_t)i) < 0.5 ? 1 : -1;
    }
  }
  for (int sp = 0; sp < 2; ++sp) {
    if ((draw_occ >> sp) & 1) {
      for (int i = TID; i < w.N; i += kThreads) w.fmark[i] = i;
      SYNC();
      if (TID == 0) {
        for (int a = 0; a < w.ne[sp]; ++a) {
          const int j = a + pick(uniform01(w.seed, w.wid, kInitOcc, 0, (uint32_t)sp, (uint32_t)a), w.N - a);
          const int t = w.fmark[a];
          w.fmark[a] = w.fmark[j];
          w.fmark[j] = t;
          w.occ[sp][a] = w.fmark[a];
        }
      }
      SYNC();
    }
  }
}

// Fresh log-weight from the current (eta, s): right stack + inverse at beta.
__global__ void __launch_bounds__(kThreads) k_fresh_weight(const WalkerDesc *__restrict__ descs, LdsPlan pl, int set_tracked) {
  const WalkerDesc &w = descs[blockIdx.x];
  Lds L = carve(pl);
  bind_mats(L, w, pl, 0);
  load_bonds(w, L, pl.bond_words);
  double la = 0.0;
  int sg = 1;
  for (int sp = 0; sp < 2; ++sp) {
    const bool res = L.phi != nullptr && (long)w.N * w.ne[sp] <= (long)pl.phi_elems;
    double *Phi = res ? L.phi : w.PhiR[sp];
    la += right_stack(w, sp, L, Phi);
    double l2;
    int s2;
    inverse_at_beta(w, sp, L, &l2, &s2);
    la += l2;
    sg *= s2;
  }
  if (TID == 0) {
    w.sc->fresh_logw = la;
    w.sc->fresh_sign = sg;
    if (set_tracked) {
      w.sc->logw = la;
      w.sc->sign = sg;
      w.sc->fock_logw[0] = w.sc->fock_logw[1] = 0.0;
      w.sc->fock_sign[0] = w.sc->fock_sign[1] = 1;
    }
  }
}

// Left stack, built backward from tau = beta: Y <- P; for slices l = L..1:
// Y <- E_K^T Y, store X'_l = Y (the left state at the flip point of slice l,
// (Phi_L(l) E_K)^T), Y <- D_l Y; at every block boundary a thin QR, LS[k-1] = Q.
// LS[n] = P.  Y stays in LDS when it fits.
// F: storage of the propagated block and of the stored left states (FP64, or
// FP32 for mixed-precision walkers); the QR and the stack LS stay FP64.
// LEAN: the plan keeps the work matrices in LDS (Ne <= 64) -- the layout of
// the common case, with fewer values live.
template <typename F, bool LEAN>
__global__ void __launch_bounds__(kThreads) k_left_stack(const WalkerDesc *__restrict__ descs, LdsPlan pl) {
  const WalkerDesc &w = descs[blockIdx.x >> 1];
  Lds L = carve<LEAN>(pl);
  if constexpr (!LEAN) bind_mats(L, w, pl, blockIdx.x & 1);
  load_bonds(w, L, pl.bond_words);
  const int N = w.N;
  {
    const int sp = blockIdx.x & 1;
    const int m = w.ne[sp];
    const bool res = L.phi != nullptr && phi_doubles((long)N * m, (int)sizeof(F)) <= (long)pl.phi_elems;
    F *Y = res ? reinterpret_cast<F *>(L.phi) : reinterpret_cast<F *>(w.X[sp]);
    F *LX = reinterpret_cast<F *>(w.LX[sp]);
    fill_P(w, sp, Y);
    copy_global(w.LS[sp] + (size_t)w.nblk * N * m, Y, (size_t)N * m);
    for (int k = w.nblk; k >= 1; --k) {
      const int l0 = (k - 1) * w.nstab + 1, l1 = min(k * w.nstab, w.L);
      for (int l = l1; l >= l0; --l) {
        apply_ekT(w, L, Y, m);
        copy_global(LX + (size_t)(l - 1) * N * m, Y, (size_t)N * m);
        apply_diag(w, Y, m, l, sp, false);
      }
      double *Q = w.LS[sp] + (size_t)(k - 1) * N * m;
      cholqr(Y, w.T[sp], Q, Y, nullptr, w.fVp + (size_t)sp * w.nblk * w.mmax * w.mmax, N, m, L, w.sc);
    }
  }
}

// Forward pass over all slices with the HS-field flips, stabilisation at
// block ends (push (Q_k, V_k)), wrap check and measurements at interior
// boundaries, and the fresh weight and inverse at tau = beta.
// F: storage of the propagated Slater blocks and of the stored left states
// (FP64, or FP32 for mixed-precision walkers).  Ratios, inverses, QR and
// weights are FP64 in both.
template <int TSEL, typename F>
__device__ __forceinline__ void forward_walker(const WalkerDesc &w, Lds &L, const LdsPlan &pl, int want_aw) {
  const int N = w.N, n = w.nblk;
  // staged-row stride: 8T for a register tile (a compile-time constant)
  const int xld = (TSEL == 1 || TSEL == 2 || TSEL == 4) ? 8 * TSEL : w.xld;
  const bool resident =
      L.phi != nullptr && phi_doubles((long)N * (w.ne[0] + w.ne[1]), (int)sizeof(F)) <= (long)pl.phi_elems;
  const uint32_t sweep = (uint32_t)(w.sc->sweep + 1);
  F *const phi[2] = {resident ? reinterpret_cast<F *>(L.phi) : reinterpret_cast<F *>(w.PhiR[0]),
                     resident ? reinterpret_cast<F *>(L.phi) + (size_t)N * w.ne[0] : reinterpret_cast<F *>(w.PhiR[1])};
  if (TID == 0) {
    Scalars *sc = w.sc;
    sc->logw += sc->fock_logw[0] + sc->fock_logw[1];
    sc->sign *= sc->fock_sign[0] * sc->fock_sign[1];
    sc->fock_logw[0] = sc->fock_logw[1] = 0.0;
    sc->fock_sign[0] = sc->fock_sign[1] = 1;
  }
  ChainAcc acc{0.0, 1.0, 0, 0, 0};
  for (int sp = 0; sp < 2; ++sp) fill_P(w, sp, phi[sp]);
  double ld_tot = 0.0;
  for (int k = 1; k <= n; ++k) {
    const int l0 = (k - 1) * w.nstab + 1;
    // fresh inverse at the flip point of the block's first slice
    for (int sp = 0; sp < 2; ++sp) {
      const int m = w.ne[sp];
      apply_diag(w, phi[sp], m, l0, sp, false);
      gram(reinterpret_cast<const F *>(w.LX[sp]) + (size_t)(l0 - 1) * N * m, m, phi[sp], m, N, L.A, L.red);
      double la;
      int sg;
      if (m > 0 && !gj_inverse(L.A, sp ? L.Ms1 : L.Ms0, m, L, &la, &sg))
        if (TID == 0) w.sc->status |= 4;
    }
    // the Ne <= 8 chain (short per-site steps) runs in the kernel's own
    // frame; the longer chains are calls
    if constexpr (TSEL == 1) forward_block_body<1, F>(w, k, sweep, L, phi, resident, xld, acc);
    else forward_block<TSEL, F>(w, k, sweep, L, phi, resident, xld, acc);
    // block end: diagonal of A from the updated inverse, kept for the wrap check
    if (k < n && want_aw)
      for (int sp = 0; sp < 2; ++sp) {
        const int m = w.ne[sp];
        const double *Ms = sp ? L.Ms1 : L.Ms0;
        const double *Xb = w.LS[sp] + (size_t)k * N * m;
        double *aw = w.Aw[sp] + (size_t)(k - 1) * N;
        for (int i = TID; i < N; i += kThreads) {
          double s = 0.0;
          for (int p = 0; p < m; ++p) {
            double t = 0.0;
            for (int q = 0; q < m; ++q) t += Ms[p * m + q] * Xb[(size_t)i * m + q];
            s += phi[sp][(size_t)i * m + p] * t;
          }
          aw[i] = s;
        }
        SYNC();
      }
    for (int sp = 0; sp < 2; ++sp) {
      const int m = w.ne[sp];
      double *Q = w.RQ[sp] + (size_t)(k - 1) * N * m;
      double *V = w.RV[sp] + (size_t)(k - 1) * m * m;
      ld_tot += cholqr(phi[sp], w.T[sp], Q, phi[sp], V, w.fVp, N, m, L, w.sc);
    }
  }
  // tau = beta: inverse of P^T Q_n and the fresh weight
  int sg_tot = 1;
  for (int sp = 0; sp < 2; ++sp) {
    double la;
    int sg;
    inverse_at_beta(w, sp, L, &la, &sg);
    ld_tot += la;
    sg_tot *= sg;
  }
  if (TID == 0) {
    Scalars *sc = w.sc;
    const double tracked = sc->logw + acc_total(acc);
    const double drift = fabs(tracked - ld_tot);
    if (drift > sc->logw_drift) sc->logw_drift = drift;
    sc->logw = ld_tot;
    sc->sign = sg_tot;
    sc->fresh_logw = ld_tot;
    sc->fresh_sign = sg_tot;
    if (!(w.flags & 2)) sc->flip_att += (long long)w.N * w.L;
    sc->flip_acc += acc.nacc;
    sc->near_ties += acc.nnear;
    sc->sweep = sweep;
  }
}

// One workgroup per walker.  TSEL >= 0: every walker of the launch has that
// chain shape (register tile T, or 0 for the LDS inverse); TSEL < 0: each
// walker's own shape is dispatched here, so walkers of different Ne share a
// launch without changing each other's arithmetic.  The walker's wall-clock
// time of the pass is recorded for the autotuner.
template <int TSEL, typename F>
__global__ void __launch_bounds__(kThreads) k_forward(const WalkerDesc *__restrict__ descs, LdsPlan pl, int want_aw) {
  const WalkerDesc &w = descs[blockIdx.x];
  const long long t0 = wall_clock64();
  constexpr bool kLean = TSEL == 1 || TSEL == 2 || TSEL == 4;
  Lds L = carve<kLean>(pl);
  if constexpr (!kLean) bind_mats(L, w, pl, 0);
  L.S = w.chunk;
  load_bonds(w, L, pl.bond_words);
  if constexpr (TSEL >= 0) {
    forward_walker<TSEL, F>(w, L, pl, want_aw);
  } else {
    switch (w.tile) {
      case 1: forward_walker<1, F>(w, L, pl, want_aw); break;
      case 2: forward_walker<2, F>(w, L, pl, want_aw); break;
      case 4: forward_walker<4, F>(w, L, pl, want_aw); break;
      case kDelayed: forward_walker<kDelayed, F>(w, L, pl, want_aw); break;
      case kMfma: forward_walker<kMfma, F>(w, L, pl, want_aw); break;
      default: forward_walker<0, F>(w, L, pl, want_aw); break;
    }
  }
  if (TID == 0) w.sc->fwd_ticks = wall_clock64() - t0;
}

// ---------------------------------------------------------------------------
// Measurements after the forward pass.  The fresh Green's function at the
// interior boundary k is fixed by the stored pair (LS[k], Q_k): LS[k] was
// built from the fields of the blocks above k before they were swept, Q_k
// from the swept fields of the blocks up to k, which is the configuration
// the sweep passes through at that boundary.  One workgroup per (walker,
// boundary) writes a partial record (estimators, wrap error); k_measure_sum
// adds the records of a walker in boundary order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int meas_slots(const WalkerDesc &w) { return w.nblk > 1 ? w.nblk - 1 : 1; }

__device__ __forceinline__ void measure_boundary(const WalkerDesc &w, Lds &L, int q) {
  const int N = w.N;
  const size_t rec = (size_t)w.nobs + 1;
  double *part = w.mpart + (size_t)q * rec;
  double *scr = w.mscr + (size_t)q * w.mscr_stride;
  MeasScratch ms;
  ms.T[0] = scr;
  ms.T[1] = scr + (size_t)N * w.mmax;
  ms.Ad[0] = scr + (size_t)2 * N * w.mmax;
  ms.Ad[1] = ms.Ad[0] + N;
  ms.Afull = ms.Ad[1] + N;
  for (int t = TID; t < (int)rec; t += kThreads) part[t] = 0.0;
  double *PR[2], *XL[2];
  const bool at_beta = w.nblk == 1;
  const int k = q + 1;
  int sg = 1;
  double wrap = 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    double *Ms = sp ? L.Ms1 : L.Ms0;
    if (at_beta) {
      PR[sp] = w.RQ[sp];
      XL[sp] = w.X[sp];
      fill_P(w, sp, XL[sp]);
      for (int t = TID; t < m * m; t += kThreads) Ms[t] = w.Minv[sp][t];
      SYNC();
      continue;
    }
    PR[sp] = w.RQ[sp] + (size_t)(k - 1) * N * m;
    XL[sp] = w.LS[sp] + (size_t)k * N * m;
    gram(XL[sp], m, PR[sp], m, N, L.A, L.red);
    double la;
    int s2 = 1;
    if (m > 0) {
      if (!gj_inverse(L.A, Ms, m, L, &la, &s2))
        if (TID == 0) w.sc->status |= 4;
      // wrap check: diagonal of A from the inverse carried through the block
      const double *aw = w.Aw[sp] + (size_t)(k - 1) * N;
      double dmax = 0.0;
      for (int i = TID; i < N; i += kThreads) {
        double s = 0.0;
        for (int p = 0; p < m; ++p) {
          double t = 0.0;
          for (int qq = 0; qq < m; ++qq) t += Ms[p * m + qq] * XL[sp][(size_t)i * m + qq];
          s += PR[sp][(size_t)i * m + p] * t;
        }
        dmax = fmax(dmax, fabs(s - aw[i]));
      }
      dmax = wg_max(dmax, L.red);
      wrap = fmax(wrap, dmax);
    }
    sg *= s2;
  }
  if (at_beta) sg = w.sc->sign;  // sign of prod det(P^T Q_n) set by this sweep's forward pass
  const double *Msp[2] = {L.Ms0, L.Ms1};
  measure_point(w, PR, XL, Msp, sg, L, part, ms);
  if (TID == 0) part[w.nobs] = wrap;
  SYNC();
}

// slots: workgroups per walker; each takes boundaries q, q + slots, ...
// (one workgroup per walker when the Ne x Ne work matrices are in device
// memory, since they are one per walker)
__global__ void __launch_bounds__(kThreads) k_measure(const WalkerDesc *__restrict__ descs, LdsPlan pl, int slots) {
  const WalkerDesc &w = descs[blockIdx.x / slots];
  Lds L = carve(pl);
  bind_mats(L, w, pl, 0);
  for (int q = blockIdx.x % slots; q < meas_slots(w); q += slots) measure_boundary(w, L, q);
}

__global__ void __launch_bounds__(kThreads) k_measure_sum(const WalkerDesc *__restrict__ descs) {
  const WalkerDesc &w = descs[blockIdx.x];
  const int slots = meas_slots(w);
  const size_t rec = (size_t)w.nobs + 1;
  for (int t = TID; t < w.nobs; t += kThreads) {
    double s = w.obs[t];
    for (int q = 0; q < slots; ++q) s += w.mpart[(size_t)q * rec + t];
    w.obs[t] = s;
  }
  if (TID == 0) {
    // wrap-versus-fresh check of the stabilisation (SM Sec. I.A): the largest
    // diagonal difference of this sweep's boundaries against the tolerance
    double sw = 0.0;
    for (int q = 0; q < slots; ++q) sw = fmax(sw, w.mpart[(size_t)q * rec + w.nobs]);
    w.sc->max_wrap = fmax(w.sc->max_wrap, sw);
    w.sc->wrap_sweep = sw;
    if (!(sw <= w.wrap_tol)) w.sc->status |= 8;
  }
}

// ---------------------------------------------------------------------------
// Particle-hole swap (removal of occupied index k, addition of site j).
// Removal (SM Sec. I.B): permutation U moving column k last, then at each
// level Givens rotations retriangulating V_1 U or V_i G_{i-1}^T; the last
// diagonal gives r_Ne, and M_perm^{-1} = G_n M^{-1} U.  Addition (SM Sec. I.A)
// on the reduced system: propagate e_j through each block, project out the
// reduced basis twice (classical Gram-Schmidt, second pass for stability),
// normalise.  Ratio r = [M_perm^{-1}]_{Ne,Ne} / r_Ne * s * prod_i rho_i.
// LDS: Ms0 = Hessenberg work, Ms1 = M_perm^{-1}, A = reduced inverse.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int perm_col(int c, int k, int ne) {
  return c < k ? c : (c < ne - 1 ? c + 1 : k);
}

// Fast path of the column propagation in the addition move: the vector lives
// in LDS and every thread owns at most kFq of its sites (i = TID + q kThreads),
// with their onsite factors cached; the fields of the next slice are loaded
// while the current one is applied, and only LDS barriers are used so that
// loads issued before the call (the level's Q rows) stay in flight.
constexpr int kFq = 4;   // sites per thread on the fast path (N <= 1024)
constexpr int kFne = 8;  // Q columns cached in registers (Ne <= 8)
template <typename F>
__device__ __forceinline__ void fock_propagate(const WalkerDesc &w, int sp, F *fw, int l0, int l1,
                                               const double (&eps)[kFq], const Lds &L) {
  const int N = w.N;
  auto v = as_lds(fw);
  int fc[kFq], fn[kFq];
  auto fields = [&](int l, int (&f)[kFq]) {
    const int8_t *srow = w.s + (size_t)(l - 1) * N;
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int i = TID + q * kThreads;
      f[q] = i < N ? srow[i] : 1;
    }
  };
  fields(l0, fc);
  for (int l = l0; l <= l1; ++l) {
    if (l < l1) fields(l + 1, fn);
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int i = TID + q * kThreads;
      const int ss = sp == 0 ? fc[q] : -fc[q];
      if (i < N) v[i] *= (F)((ss > 0 ? w.elam : w.emlam) * eps[q]);
    }
    lds_sync();
    apply_ek(w, L, fw, 1);
#pragma unroll
    for (int q = 0; q < kFq; ++q) fc[q] = fn[q];
  }
}

// The column's checkerboard passes with the bonds of each thread held in
// registers: bond TID + u * kThreads of colour c, packed as
// i | j << 10 | coefficient index << 20 (or -1).  Valid for N <= 1024 (so a
// colour, whose bonds are site-disjoint, has at most 2 kThreads bonds), at
// most kFcol colours, and bond tables in LDS.
constexpr int kFcol = 8;
struct FockBonds {
  int w[kFcol][2];
};
__device__ __forceinline__ bool fock_bonds(const WalkerDesc &w, const Lds &L, FockBonds &fb) {
  if (!(L.bonds_ok && L.cs && w.N <= kFq * kThreads && w.ncol <= kFcol)) return false;
  const BondSrc bs = bond_src(L, w);
#pragma unroll
  for (int c = 0; c < kFcol; ++c)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int v = -1;
      if (c < w.ncol) {
        const int b = bs.cs[c] + TID + u * kThreads;
        if (b < bs.cs[c + 1]) {
          const int ij = bs.bij[b];
          v = (ij & 0xffff) | (int)(((unsigned)ij >> 16) << 10) | ((int)bs.bci[b] << 20);
        }
      }
      fb.w[c][u] = v;
    }
  return true;
}
// one colour pass over the LDS column v (same arithmetic as colour_pass_t),
// without branches: a thread with no bond in a slot reads and writes its own
// dummy word, so that every load is issued before the first store
template <typename P>
__device__ __forceinline__ void fock_pass(const int (&wc)[2], P v, P dummy, const lds_f64 *coef) {
  using E = typename Elem<P>::T;
  P pi[2], pj[2];
  E xi[2], xj[2], d[2], o[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const bool ok = wc[u] >= 0;
    const int a = ok ? wc[u] : 0;
    pi[u] = ok ? v + (a & 1023) : dummy;
    pj[u] = ok ? v + ((a >> 10) & 1023) : dummy;
    const int ci = a >> 20;
    xi[u] = *pi[u];
    xj[u] = *pj[u];
    d[u] = (E)coef[2 * ci];
    o[u] = (E)coef[2 * ci + 1];
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    *pi[u] = d[u] * xi[u] + o[u] * xj[u];
    *pj[u] = o[u] * xi[u] + d[u] * xj[u];
  }
  lds_sync();
}
// The fields of the level's slices (at most kFsl) for the thread's kFq sites
// are read once, as bits (site q of slice l0 + t at bit kFq t + q).
constexpr int kFsl = 16;
// the first colour pass of a slice with the slice's diagonal factors folded
// in: each end of a bond is scaled (as the diagonal pass scales it) before
// the rotation; used when that colour's bonds cover every site once
template <typename P>
__device__ __forceinline__ void fock_pass_diag(const int (&wc)[2], P v, P dummy, const lds_f64 *coef,
                                               const double (&fac)[4]) {
  using E = typename Elem<P>::T;
  P pi[2], pj[2];
  E xi[2], xj[2], d[2], o[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const bool ok = wc[u] >= 0;
    const int a = ok ? wc[u] : 0;
    pi[u] = ok ? v + (a & 1023) : dummy;
    pj[u] = ok ? v + ((a >> 10) & 1023) : dummy;
    const int ci = a >> 20;
    xi[u] = *pi[u];
    xj[u] = *pj[u];
    d[u] = (E)coef[2 * ci];
    o[u] = (E)coef[2 * ci + 1];
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const E si = xi[u] * (E)fac[2 * u], sj = xj[u] * (E)fac[2 * u + 1];
    *pi[u] = d[u] * si + o[u] * sj;
    *pj[u] = o[u] * si + d[u] * sj;
  }
  lds_sync();
}
template <typename F>
__device__ __forceinline__ void fock_propagate_cb(const WalkerDesc &w, int sp, F *fw, int l0, int l1,
                                                  const double (&eps)[kFq], const Lds &L, const FockBonds &fb) {
  const int N = w.N, ncol = w.ncol, nsl = l1 - l0 + 1;
  const double elam = w.elam, emlam = w.emlam;
  const lds_f64 *coef = as_lds(L.bonds);
  auto v = as_lds(fw);
  auto dummy = as_lds(reinterpret_cast<F *>(L.red + TID));
  // The first colour's bonds cover every site once (N / 2 disjoint bonds):
  // the diagonal factors are folded into that pass, taken at the four ends of
  // the thread's two bonds of it.
  if (N % 2 == 0 && L.cs[ncol] - L.cs[ncol - 1] == N / 2) {
    int w0[2] = {-1, -1};   // the first colour's bond words (constant indices keep fb in registers)
#pragma unroll
    for (int c = 0; c < kFcol; ++c)
      if (c == ncol - 1) {
        w0[0] = fb.w[c][0];
        w0[1] = fb.w[c][1];
      }
    int site[4];
    bool real[4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool ok = w0[u] >= 0;
      const int a = ok ? w0[u] : 0;
      site[2 * u] = a & 1023;
      site[2 * u + 1] = (a >> 10) & 1023;
      real[2 * u] = real[2 * u + 1] = ok;
    }
    int8_t f[kFsl][4];
    double epe[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) epe[e] = w.eps_fac[site[e]];
#pragma unroll
    for (int t = 0; t < kFsl; ++t) {
      const int8_t *srow = w.s + (size_t)(l0 - 1 + (t < nsl ? t : nsl - 1)) * N;
#pragma unroll
      for (int e = 0; e < 4; ++e) f[t][e] = srow[site[e]];
    }
    unsigned long long bits = 0;
#pragma unroll
    for (int t = 0; t < kFsl; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (t < nsl && real[e] && f[t][e] > 0) bits |= 1ull << (4 * t + e);
    for (int t = 0; t < nsl; ++t) {
      double fac[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool up = (bits >> (4 * t + e)) & 1ull;
        const int ss = (sp == 0) == up ? 1 : -1;
        fac[e] = (ss > 0 ? elam : emlam) * epe[e];
      }
      // E_K: colour ncol - 1 acts first, with D folded in
      fock_pass_diag(w0, v, dummy, coef, fac);
#pragma unroll
      for (int c = kFcol - 2; c >= 0; --c)
        if (c < ncol - 1) fock_pass(fb.w[c], v, dummy, coef);
    }
    return;
  }
  // every load is issued (rows and sites clamped into range) before any is used
  int8_t f[kFsl][kFq];
#pragma unroll
  for (int t = 0; t < kFsl; ++t) {
    const int8_t *srow = w.s + (size_t)(l0 - 1 + (t < nsl ? t : nsl - 1)) * N;
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int i = TID + q * kThreads;
      f[t][q] = srow[i < N ? i : 0];
    }
  }
  unsigned long long bits = 0;
#pragma unroll
  for (int t = 0; t < kFsl; ++t)
#pragma unroll
    for (int q = 0; q < kFq; ++q)
      if (t < nsl && TID + q * kThreads < N && f[t][q] > 0) bits |= 1ull << (kFq * t + q);
  for (int t = 0; t < nsl; ++t) {
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int i = TID + q * kThreads;
      const bool up = (bits >> (kFq * t + q)) & 1ull;
      const int ss = (sp == 0) == up ? 1 : -1;
      if (i < N) v[i] *= (F)((ss > 0 ? elam : emlam) * eps[q]);
    }
    lds_sync();
    // E_K: colour ncol - 1 acts first
#pragma unroll
    for (int c = kFcol - 1; c >= 0; --c)
      if (c < ncol) fock_pass(fb.w[c], v, dummy, coef);
  }
}

// Projections of the addition against a level's basis Q (N x ne, row-major,
// device memory) when the rows are not cached in registers.  The lanes of a
// wave run across the columns of a row, two columns per lane (16-byte loads
// when ne is even), ne2 = ceil(ne / 2) rounded up to a power of two (at most
// 64) lanes per row, 64 / ne2 rows side by side; above 128 columns a lane
// takes the pairs c, c + 64, ...  Sixteen row groups are in flight per lane
// (64 KiB per workgroup), since a level's basis comes from device memory.
// Sums are taken in a fixed order (xor butterflies, then the four waves in
// order), so the result does not depend on timing.
struct QMap {
  int ne2, rpi, rsub, col, ncq;
};
__device__ __forceinline__ QMap qmap(int ne) {
  QMap q;
  const int np = (ne + 1) >> 1;
  q.ne2 = 1;
  while (q.ne2 < np && q.ne2 < 64) q.ne2 <<= 1;
  q.rpi = 64 / q.ne2;
  const int lane = TID & 63;
  q.rsub = lane / q.ne2;
  q.col = lane - q.rsub * q.ne2;
  q.ncq = (np + 63) >> 6;
  return q;
}
// The pair of columns (2 cp, 2 cp + 1) of row i, loaded unconditionally
// from indices clamped into the block (so that no wait separates the loads
// of a round); qzero() then zeroes what lies outside.  VEC: one 16-byte load
// (ne even).
template <bool VEC>
__device__ __forceinline__ void qpair(gc_f64 *Q, int ne, int N, int i, int cp, double &x0, double &x1) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) const d2v gc_d2;
  const int c0 = 2 * cp;
  const size_t ic = (size_t)min(i, N - 1) * ne;
  if constexpr (VEC) {
    const d2v v = *(gc_d2 *)(Q + ic + min(c0, ne - 2));
    x0 = v[0];
    x1 = v[1];
  } else {
    x0 = Q[ic + min(c0, ne - 1)];
    x1 = Q[ic + min(c0 + 1, ne - 1)];
  }
}
__device__ __forceinline__ void qzero(int ne, int N, int i, int cp, double &x0, double &x1) {
  const int c0 = 2 * cp;
  const bool ok = i < N && c0 < ne;
  x0 = ok ? x0 : 0.0;
  x1 = (ok && c0 + 1 < ne) ? x1 : 0.0;
}
constexpr int kQR = 16;   // row groups in flight per lane
// y[a] = sum_i Q[i][a] f[i] for a < ne, into y (LDS)
template <bool VEC, typename PF>
__device__ __forceinline__ void fock_qt_t(const double *Qg, int ne, int N, PF f, double *y, double *red) {
  gc_f64 *Q = as_global(Qg);
  const QMap mp = qmap(ne);
  const int wave = TID >> 6, step = 4 * mp.rpi;
  for (int c = 0; c < mp.ncq; ++c) {
    const int cp = mp.col + 64 * c;
    double a0 = 0.0, a1 = 0.0;
    for (int i0 = wave * mp.rpi; i0 < N; i0 += kQR * step) {
      double x0[kQR], x1[kQR], fv[kQR];
#pragma unroll
      for (int u = 0; u < kQR; ++u) qpair<VEC>(Q, ne, N, i0 + u * step + mp.rsub, cp, x0[u], x1[u]);
      __builtin_amdgcn_sched_barrier(0);   // every load of the round goes out before the first use
#pragma unroll
      for (int u = 0; u < kQR; ++u) qzero(ne, N, i0 + u * step + mp.rsub, cp, x0[u], x1[u]);
#pragma unroll
      for (int u = 0; u < kQR; ++u) {
        const int ii = i0 + u * step + mp.rsub;
        const double v = (double)f[min(ii, N - 1)];
        fv[u] = ii < N ? v : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kQR; ++u) {
        a0 = fma(x0[u], fv[u], a0);
        a1 = fma(x1[u], fv[u], a1);
      }
    }
    // sum over the rows a wave reads side by side, then over the waves
    for (int m = mp.ne2; m < 64; m <<= 1) {
      a0 += __shfl_xor(a0, m);
      a1 += __shfl_xor(a1, m);
    }
    if (mp.ne2 == 64) {
      // 64 lanes per row: the even columns, then the odd ones, through red
      if (mp.rsub == 0) red[wave * 64 + mp.col] = a0;
      SYNC();
      const int cc = 128 * c + 2 * TID;
      if (TID < 64 && cc < ne) y[cc] = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
      SYNC();
      if (mp.rsub == 0) red[wave * 64 + mp.col] = a1;
      SYNC();
      if (TID < 64 && cc + 1 < ne) y[cc + 1] = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
      SYNC();
    } else {
      if (mp.rsub == 0) {
        red[wave * 64 + mp.col] = a0;
        red[wave * 64 + 32 + mp.col] = a1;   // col < 32 here
      }
      SYNC();
      if (TID < mp.ne2) {
        const int cc = 2 * TID;
        const double s0 = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
        const double s1 = (red[32 + TID] + red[96 + TID]) + (red[160 + TID] + red[224 + TID]);
        if (cc < ne) y[cc] = s0;
        if (cc + 1 < ne) y[cc + 1] = s1;
      }
      SYNC();
    }
  }
}
// f[i] -= sum_a Q[i][a] z[a] (z: ne entries in LDS)
template <bool VEC, typename PF>
__device__ __forceinline__ void fock_sub_t(const double *Qg, int ne, int N, PF f, const double *z) {
  gc_f64 *Q = as_global(Qg);
  const lds_f64 *zl = as_lds(z);
  const QMap mp = qmap(ne);
  const int wave = TID >> 6, step = 4 * mp.rpi;
  double z0[4], z1[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cc = 2 * (mp.col + 64 * c);
    z0[c] = (c < mp.ncq && cc < ne) ? zl[cc] : 0.0;
    z1[c] = (c < mp.ncq && cc + 1 < ne) ? zl[cc + 1] : 0.0;
  }
  for (int i0 = wave * mp.rpi; i0 < N; i0 += kQR * step) {
    double sm[kQR];
#pragma unroll
    for (int u = 0; u < kQR; ++u) sm[u] = 0.0;
    for (int c = 0; c < mp.ncq; ++c) {
      double x0[kQR], x1[kQR];
#pragma unroll
      for (int u = 0; u < kQR; ++u) qpair<VEC>(Q, ne, N, i0 + u * step + mp.rsub, mp.col + 64 * c, x0[u], x1[u]);
      __builtin_amdgcn_sched_barrier(0);   // every load of the round goes out before the first use
#pragma unroll
      for (int u = 0; u < kQR; ++u) qzero(ne, N, i0 + u * step + mp.rsub, mp.col + 64 * c, x0[u], x1[u]);
      const double zc0 = c == 0 ? z0[0] : c == 1 ? z0[1] : c == 2 ? z0[2] : z0[3];
      const double zc1 = c == 0 ? z1[0] : c == 1 ? z1[1] : c == 2 ? z1[2] : z1[3];
#pragma unroll
      for (int u = 0; u < kQR; ++u) sm[u] = fma(x1[u], zc1, fma(x0[u], zc0, sm[u]));
    }
    // row sums over the row's lanes (every lane of the row ends with them)
    for (int m = 1; m < mp.ne2; m <<= 1)
#pragma unroll
      for (int u = 0; u < kQR; ++u) sm[u] += __shfl_xor(sm[u], m);
    if (mp.col == 0)
#pragma unroll
      for (int u = 0; u < kQR; ++u) {
        const int ii = i0 + u * step + mp.rsub;
        if (ii < N) f[ii] -= sm[u];
      }
  }
}

// One pass over Q for the second Gram-Schmidt pass: f[i] -= sum_a Q[i][a] z[a]
// (as fock_sub), and y[a] = sum_i Q[i][a] f[i] of the updated f (as fock_qt),
// from the same loaded rows.  Rows, lanes and summation order are those of
// the two separate passes, so y and f come out bit-identical to them.  For
// ne <= 128 (one column pair per lane).
constexpr int kQF = 8;   // row groups in flight per lane in the fused pass (it holds four arrays)
template <bool VEC, typename PF>
__device__ __forceinline__ void fock_subqt_t(const double *Qg, int ne, int N, PF f, const double *z, double *y,
                                             double *red) {
  using FE = typename Elem<PF>::T;
  gc_f64 *Q = as_global(Qg);
  const lds_f64 *zl = as_lds(z);
  const QMap mp = qmap(ne);
  const int wave = TID >> 6, step = 4 * mp.rpi;
  const int cc = 2 * mp.col;
  const double zc0 = cc < ne ? zl[cc] : 0.0, zc1 = cc + 1 < ne ? zl[cc + 1] : 0.0;
  double a0 = 0.0, a1 = 0.0;
  for (int i0 = wave * mp.rpi; i0 < N; i0 += kQF * step) {
    double x0[kQF], x1[kQF], fo[kQF], sm[kQF];
#pragma unroll
    for (int u = 0; u < kQF; ++u) qpair<VEC>(Q, ne, N, i0 + u * step + mp.rsub, mp.col, x0[u], x1[u]);
#pragma unroll
    for (int u = 0; u < kQF; ++u) fo[u] = (double)f[min(i0 + u * step + mp.rsub, N - 1)];
    __builtin_amdgcn_sched_barrier(0);   // every load of the round goes out before the first use
#pragma unroll
    for (int u = 0; u < kQF; ++u) qzero(ne, N, i0 + u * step + mp.rsub, mp.col, x0[u], x1[u]);
#pragma unroll
    for (int u = 0; u < kQF; ++u) sm[u] = fma(x1[u], zc1, fma(x0[u], zc0, 0.0));
    for (int m = 1; m < mp.ne2; m <<= 1)
#pragma unroll
      for (int u = 0; u < kQF; ++u) sm[u] += __shfl_xor(sm[u], m);
#pragma unroll
    for (int u = 0; u < kQF; ++u) {
      const int ii = i0 + u * step + mp.rsub;
      FE nf = (FE)fo[u];
      nf -= sm[u];
      if (mp.col == 0 && ii < N) f[ii] = nf;
      const double fv = ii < N ? (double)nf : 0.0;
      a0 = fma(x0[u], fv, a0);
      a1 = fma(x1[u], fv, a1);
    }
  }
  for (int m = mp.ne2; m < 64; m <<= 1) {
    a0 += __shfl_xor(a0, m);
    a1 += __shfl_xor(a1, m);
  }
  if (mp.ne2 == 64) {
    if (mp.rsub == 0) red[wave * 64 + mp.col] = a0;
    SYNC();
    if (TID < 64 && 2 * TID < ne) y[2 * TID] = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
    SYNC();
    if (mp.rsub == 0) red[wave * 64 + mp.col] = a1;
    SYNC();
    if (TID < 64 && 2 * TID + 1 < ne)
      y[2 * TID + 1] = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
    SYNC();
  } else {
    if (mp.rsub == 0) {
      red[wave * 64 + mp.col] = a0;
      red[wave * 64 + 32 + mp.col] = a1;
    }
    SYNC();
    if (TID < mp.ne2) {
      const double s0 = (red[TID] + red[64 + TID]) + (red[128 + TID] + red[192 + TID]);
      const double s1 = (red[32 + TID] + red[96 + TID]) + (red[160 + TID] + red[224 + TID]);
      if (2 * TID < ne) y[2 * TID] = s0;
      if (2 * TID + 1 < ne) y[2 * TID + 1] = s1;
    }
    SYNC();
  }
}
template <typename PF>
__device__ __forceinline__ void fock_subqt(const double *Q, int ne, int N, PF f, const double *z, double *y,
                                           double *red) {
  if ((ne & 1) == 0) fock_subqt_t<true>(Q, ne, N, f, z, y, red);
  else fock_subqt_t<false>(Q, ne, N, f, z, y, red);
}

template <typename PF>
__device__ __forceinline__ void fock_qt(const double *Q, int ne, int N, PF f, double *y, double *red) {
  if ((ne & 1) == 0) fock_qt_t<true>(Q, ne, N, f, y, red);
  else fock_qt_t<false>(Q, ne, N, f, y, red);
}
template <typename PF>
__device__ __forceinline__ void fock_sub(const double *Q, int ne, int N, PF f, const double *z) {
  if ((ne & 1) == 0) fock_sub_t<true>(Q, ne, N, f, z);
  else fock_sub_t<false>(Q, ne, N, f, z);
}

// returns accepted (uniform); *log_abs_r / *sign_r in scal.  F: storage of
// the propagated column (FP32 for mixed-precision walkers); projections,
// norms, the stored columns q_i and every ratio are FP64.
// The Givens coefficients of the removal are kept in LDS as well (the last
// two levels in uw, the current level of the addition in vec[6..7]) so that
// the serial rotations of thread 0 read no device memory.
template <typename F>
__device__ bool swap_move(const WalkerDesc &w, int sp, int k, int j, double xacc, bool commit,
                          Lds &L, F *fw, double *ratio_out) {
  const int N = w.N, ne = w.ne[sp], m = ne - 1, n = w.nblk, mm = w.mmax;
  // per-spin Fock scratch
  double *const fq = w.fq + (size_t)sp * n * N;
  double *const fVp = w.fVp + (size_t)sp * n * mm * mm;
  double *const fgc = w.fgc + (size_t)sp * n * mm;
  double *const fgs = w.fgs + (size_t)sp * n * mm;
  double *const fv = w.fv + (size_t)sp * n * mm;
  double *const frho = w.frho + (size_t)sp * n;
  double *H = L.Ms0, *Mp = L.Ms1, *Mred = L.A;
  const int vs = L.vs;
  double *y = L.vec, *z = L.vec + vs, *vsum = L.vec + 2 * vs, *acol = L.vec + 3 * vs, *brow = L.vec + 4 * vs,
         *tv = L.vec + 5 * vs, *gcl = L.vec + 6 * vs, *gsl = L.vec + 7 * vs;
  // removal coefficients of level lvl in LDS: cosines at uw + (lvl & 1) vs, sines 2 vs further
  auto gcb = [&](int lvl) { return L.uw + (lvl & 1) * vs; };
  auto gsb = [&](int lvl) { return L.uw + (2 + (lvl & 1)) * vs; };
  // scal[20] log_rne, [21] sign_rne, [22] zero flag, [23] log_rho
  if (TID == 0) { L.scal[20] = 0.0; L.scal[21] = 1.0; L.scal[22] = 0.0; L.scal[23] = 0.0; }
  SYNC();
  // ---- removal ----
  for (int lvl = 0; lvl < n; ++lvl) {
    const double *V = w.RV[sp] + (size_t)lvl * ne * ne;
    if (lvl == 0) {
      for (int t = TID; t < ne * ne; t += kThreads) {
        const int r = t / ne, c = t % ne;
        H[t] = V[r * ne + perm_col(c, k, ne)];
      }
      SYNC();
    } else {
      // H = V_i G_{i-1}^T: every row takes the previous level's column
      // rotations in order, one thread per row (no barrier between them)
      const double *gc = gcb(lvl - 1), *gs = gsb(lvl - 1);
      for (int row = TID; row < ne; row += kThreads) {
        gc_f64 *vr = as_global(V + (size_t)row * ne);
        double *hr = H + (size_t)row * ne;
        for (int a = 0; a < k; ++a) hr[a] = vr[a];
        double carry = vr[k];
        // sixteen loads of the row in flight before their rotations
        for (int r0 = k; r0 <= ne - 2; r0 += 16) {
          const int nr = min(16, ne - 1 - r0);
          double b[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) b[u] = u < nr ? vr[r0 + 1 + u] : 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (u < nr) {
              const double cc = gc[r0 + u], ss = gs[r0 + u];
              hr[r0 + u] = cc * carry + ss * b[u];
              carry = -ss * carry + cc * b[u];
            }
        }
        hr[ne - 1] = carry;
      }
      SYNC();
    }
    double *gc = fgc + (size_t)lvl * mm, *gs = fgs + (size_t)lvl * mm;
    // Givens retriangulation of the Hessenberg part (rows k..ne-1) by wave 0:
    // the carried row r and the next row r + 1 in registers (lane l owns
    // columns l, l + 64, ...), the pivot pair broadcast by readlane
    if (TID < 64 && k <= ne - 2) {
      const int lane = TID;
      double carry[4], nxt[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = lane + 64 * q;
        carry[q] = col < ne ? H[k * ne + col] : 0.0;
      }
      for (int r = k; r <= ne - 2; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = lane + 64 * q;
          nxt[q] = col < ne ? H[(r + 1) * ne + col] : 0.0;
        }
        const int qr = r >> 6, lr = r & 63;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q == qr) {
            a = lane_read(carry[q], lr);
            b = lane_read(nxt[q], lr);
          }
        const double hh = hypot(a, b);
        double cc = 1.0, ss = 0.0;
        if (hh != 0.0) { cc = a / hh; ss = b / hh; }
        if (lane == 0) {
          gc[r] = cc;
          gs[r] = ss;
          gcb(lvl)[r] = cc;
          gsb(lvl)[r] = ss;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = lane + 64 * q;
          const double u = carry[q], d = nxt[q];
          if (col < ne) H[r * ne + col] = cc * u + ss * d;
          carry[q] = col == r ? 0.0 : -ss * u + cc * d;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = lane + 64 * q;
        if (col < ne) H[(ne - 1) * ne + col] = carry[q];
      }
    }
    SYNC();
    double *Vp = fVp + (size_t)lvl * mm * mm;
    for (int t = TID; t < ne * ne; t += kThreads) Vp[t] = H[t];
    if (TID == 0) {
      const double last = H[(ne - 1) * ne + (ne - 1)];
      L.scal[20] += log(fabs(last));
      if (last < 0.0) L.scal[21] = -L.scal[21];
      if (last == 0.0) L.scal[22] = 1.0;
    }
    SYNC();
  }
  // M_perm^{-1} = G_n M^{-1} U  (B as work)
  {
    double *Tm = L.B;
    for (int t = TID; t < ne * ne; t += kThreads) Tm[t] = w.Minv[sp][t];
    SYNC();
    // rows rotated in order, one thread per column (no barrier between them)
    const double *gc = gcb(n - 1), *gs = gsb(n - 1);
    for (int col = TID; col < ne; col += kThreads) {
      double carry = Tm[k * ne + col];
      for (int r0 = k; r0 <= ne - 2; r0 += 16) {
        const int nr = min(16, ne - 1 - r0);
        double b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) b[u] = u < nr ? Tm[(r0 + 1 + u) * ne + col] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (u < nr) {
            const double cc = gc[r0 + u], ss = gs[r0 + u];
            Tm[(r0 + u) * ne + col] = cc * carry + ss * b[u];
            carry = -ss * carry + cc * b[u];
          }
      }
      Tm[(ne - 1) * ne + col] = carry;
    }
    SYNC();
    for (int t = TID; t < ne * ne; t += kThreads) {
      const int r = t / ne, c = t % ne;
      Mp[t] = Tm[r * ne + perm_col(c, k, ne)];
    }
    SYNC();
  }
  const double mlast = Mp[(ne - 1) * ne + (ne - 1)];
  if (TID == 0 && mlast == 0.0) L.scal[22] = 1.0;
  for (int t = TID; t < m * m; t += kThreads) {
    const int a = t / m, b = t % m;
    Mred[t] = Mp[a * ne + b] - Mp[a * ne + (ne - 1)] * Mp[(ne - 1) * ne + b] / mlast;
  }
  SYNC();
  const double log_rem = log(fabs(mlast)) - L.scal[20];
  const double sign_rem = (mlast < 0.0 ? -1.0 : 1.0) * L.scal[21];
  // ---- addition ----
  if (L.scal[22] == 0.0) {
    for (int i = TID; i < N; i += kThreads) fw[i] = (F)((i == j) ? 1 : 0);
    SYNC();
    const bool fast = in_lds(fw) && N <= kFq * kThreads;
    const bool qcache = fast && ne <= kFne;
    FockBonds fb;
    const bool cb = fast && w.nstab <= kFsl && fock_bonds(w, L, fb);
    double eps_r[kFq];
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int i = TID + q * kThreads;
      eps_r[q] = (fast && i < N) ? w.eps_fac[i] : 1.0;
    }
    for (int lvl = 0; lvl < n; ++lvl) {
      const int l0 = lvl * w.nstab + 1, l1 = min((lvl + 1) * w.nstab, w.L);
      const double *Q = w.RQ[sp] + (size_t)lvl * N * ne;
      // the level's Q rows of this thread's sites, loaded under the propagation
      double qr[kFq][kFne];
      if (qcache) {
#pragma unroll
        for (int q = 0; q < kFq; ++q) {
          const int i = TID + q * kThreads;
#pragma unroll
          for (int a = 0; a < kFne; ++a) qr[q][a] = (i < N && a < ne) ? Q[(size_t)i * ne + a] : 0.0;
        }
      }
      // this level's rotation coefficients, loaded under the propagation
      double gcr = 0.0, gsr = 0.0;
      if (TID < ne) {
        gcr = fgc[(size_t)lvl * mm + TID];
        gsr = fgs[(size_t)lvl * mm + TID];
      }
      if (cb) {
        fock_propagate_cb(w, sp, fw, l0, l1, eps_r, L, fb);
      } else if (fast) {
        fock_propagate(w, sp, fw, l0, l1, eps_r, L);
      } else {
        for (int l = l0; l <= l1; ++l) {
          apply_diag(w, fw, 1, l, sp, false);
          apply_ek(w, L, fw, 1);
        }
      }
      if (TID < ne) {
        gcl[TID] = gcr;
        gsl[TID] = gsr;
      }
      const double *gc = gcl, *gs = gsl;
      for (int a = TID; a < vs; a += kThreads) vsum[a] = 0.0;
      SYNC();
      // the second pass's projection rides on the first pass's subtraction
      // (fock_subqt: one read of Q_i fewer per level)
      const bool fuse = !qcache && ne <= 128;
      for (int pass = 0; pass < 2 && m > 0; ++pass) {
        if (fuse && pass == 1) {
          // y holds Q^T w already
        } else if (qcache) {
          // y = Q^T w: per-thread partial sums over own rows, then a block sum
          double yp[kFne];
#pragma unroll
          for (int a = 0; a < kFne; ++a) yp[a] = 0.0;
#pragma unroll
          for (int q = 0; q < kFq; ++q) {
            const int i = TID + q * kThreads;
            const double f = (double)as_lds(fw)[i < N ? i : 0];
#pragma unroll
            for (int a = 0; a < kFne; ++a) yp[a] += qr[q][a] * (i < N ? f : 0.0);
          }
#pragma unroll
          for (int a = 0; a < kFne; ++a) yp[a] = wave_sum_d(yp[a]);
          if ((TID & 63) == 0)
#pragma unroll
            for (int a = 0; a < kFne; ++a) L.red[(TID >> 6) * kFne + a] = yp[a];
          SYNC();
          if (TID < ne)
            y[TID] = (L.red[TID] + L.red[kFne + TID]) + (L.red[2 * kFne + TID] + L.red[3 * kFne + TID]);
          SYNC();
        } else if (in_lds(fw)) {
          fock_qt(Q, ne, N, as_lds(fw), y, L.red);  // y = Q^T w
        } else {
          fock_qt(Q, ne, N, fw, y, L.red);
        }
        if (TID == 0 && ne <= kFne) {
          // the same steps on register copies (ne <= kFne): one LDS round trip
          double yr[kFne], cr[kFne], sr[kFne];
#pragma unroll
          for (int a = 0; a < kFne; ++a) {
            yr[a] = a < ne ? as_lds(y)[a] : 0.0;
            cr[a] = a < ne ? as_lds(gc)[a] : 1.0;
            sr[a] = a < ne ? as_lds(gs)[a] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < kFne - 1; ++r)
            if (r >= k && r <= ne - 2) {
              const double a = yr[r], b = yr[r + 1];
              yr[r] = cr[r] * a + sr[r] * b;
              yr[r + 1] = -sr[r] * a + cr[r] * b;
            }
#pragma unroll
          for (int a = 0; a < kFne; ++a) {
            yr[a] = a < m ? yr[a] : 0.0;
            if (a < m) as_lds(vsum)[a] += yr[a];
          }
#pragma unroll
          for (int r = kFne - 2; r >= 0; --r)
            if (r >= k && r <= ne - 2) {
              const double a = yr[r], b = yr[r + 1];
              yr[r] = cr[r] * a - sr[r] * b;
              yr[r + 1] = sr[r] * a + cr[r] * b;
            }
#pragma unroll
          for (int a = 0; a < kFne; ++a)
            if (a < ne) as_lds(z)[a] = yr[a];
        } else if (TID == 0) {
          for (int r = k; r <= ne - 2; ++r) {
            const double a = y[r], b = y[r + 1];
            y[r] = gc[r] * a + gs[r] * b;
            y[r + 1] = -gs[r] * a + gc[r] * b;
          }
          for (int a = 0; a < ne; ++a) z[a] = a < m ? y[a] : 0.0;
          for (int a = 0; a < m; ++a) vsum[a] += z[a];
          for (int r = ne - 2; r >= k; --r) {
            const double a = z[r], b = z[r + 1];
            z[r] = gc[r] * a - gs[r] * b;
            z[r + 1] = gs[r] * a + gc[r] * b;
          }
        }
        SYNC();
        if (qcache) {
#pragma unroll
          for (int q = 0; q < kFq; ++q) {
            const int i = TID + q * kThreads;
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < kFne; ++a)
              if (a < ne) s += qr[q][a] * z[a];
            if (i < N) fw[i] -= s;
          }
        } else if (fuse && pass == 0) {
          if (in_lds(fw)) fock_subqt(Q, ne, N, as_lds(fw), z, y, L.red);
          else fock_subqt(Q, ne, N, fw, z, y, L.red);
        } else if (in_lds(fw)) {
          fock_sub(Q, ne, N, as_lds(fw), z);
        } else {
          fock_sub(Q, ne, N, fw, z);
        }
        SYNC();
      }
      double nrm = 0.0;
      for (int i = TID; i < N; i += kThreads) nrm += (double)fw[i] * (double)fw[i];
      {
        // block sum: wave sums by DPP, then the four waves in a fixed order
        nrm = wave_sum_d(nrm);
        SYNC();
        if ((TID & 63) == 0) L.red[TID >> 6] = nrm;
        SYNC();
        nrm = sqrt((L.red[0] + L.red[1]) + (L.red[2] + L.red[3]));
      }
      if (!(nrm > 1e-300)) {
        if (TID == 0) L.scal[22] = 1.0;
        SYNC();
        break;
      }
      double *q = fq + (size_t)lvl * N;
      for (int i = TID; i < N; i += kThreads) {
        const double v = (double)fw[i] / nrm;
        q[i] = v;
        fw[i] = (F)v;
      }
      if (TID == 0) {
        for (int a = 0; a < m; ++a) fv[(size_t)lvl * mm + a] = vsum[a];
        frho[lvl] = nrm;
        L.scal[23] += log(nrm);
      }
      SYNC();
    }
  }
  bool accepted = false;
  double ratio = 0.0;
  if (L.scal[22] == 0.0) {
    const double *Qn = w.RQ[sp] + (size_t)(n - 1) * N * ne;
    const double *qn = fq + (size_t)(n - 1) * N;
    const int *occ = w.occ[sp];
    if (TID == 0) {
      const double *gc = gcb(n - 1), *gs = gsb(n - 1);
      for (int a = 0; a < ne; ++a) tv[a] = Qn[(size_t)j * ne + a];
      for (int r = k; r <= ne - 2; ++r) {
        const double a = tv[r], b = tv[r + 1];
        tv[r] = gc[r] * a + gs[r] * b;
        tv[r + 1] = -gs[r] * a + gc[r] * b;
      }
    }
    SYNC();
    for (int a = TID; a < m; a += kThreads) {
      double s = 0.0;
      for (int b = 0; b < m; ++b) s += Mred[a * m + b] * qn[occ[perm_col(b, k, ne)]];
      acol[a] = s;
    }
    for (int b = TID; b < m; b += kThreads) {
      double s = 0.0;
      for (int a = 0; a < m; ++a) s += tv[a] * Mred[a * m + b];
      brow[b] = s;
    }
    SYNC();
    if (TID == 0) {
      double sch = qn[j];
      for (int a = 0; a < m; ++a) sch -= tv[a] * acol[a];
      L.scal[26] = sch;
    }
    SYNC();
    const double sch = L.scal[26];
    if (sch != 0.0) {
      const double lr = log_rem + log(fabs(sch)) + L.scal[23];
      const double sr = sign_rem * (sch < 0.0 ? -1.0 : 1.0);
      ratio = sr * exp(lr);
      accepted = xacc < exp(lr);
      if (accepted && commit) {
        for (int lvl = 0; lvl < n; ++lvl) {
          double *Q = w.RQ[sp] + (size_t)lvl * N * ne;
          if (TID < ne) {
            gcl[TID] = fgc[(size_t)lvl * mm + TID];
            gsl[TID] = fgs[(size_t)lvl * mm + TID];
          }
          SYNC();
          const lds_f64 *gc = as_lds(gcl), *gs = as_lds(gsl);
          const double *q = fq + (size_t)lvl * N;
          // rows rotated by the level's Givens sequence (the removed column
          // ends last and is replaced by q_i); sixteen loads of a row are in
          // flight before its rotations and stores
          for (int i = TID; i < N; i += kThreads) {
            double *row = Q + (size_t)i * ne;
            double carry = row[k];
            for (int r0 = k; r0 <= ne - 2; r0 += 16) {
              const int nr = min(16, ne - 1 - r0);
              double b[16];
#pragma unroll
              for (int u = 0; u < 16; ++u) b[u] = u < nr ? row[r0 + 1 + u] : 0.0;
#pragma unroll
              for (int u = 0; u < 16; ++u)
                if (u < nr) {
                  const double cc = gc[r0 + u], ss = gs[r0 + u];
                  row[r0 + u] = cc * carry + ss * b[u];
                  carry = -ss * carry + cc * b[u];
                }
            }
            row[ne - 1] = q[i];
          }
          double *V = w.RV[sp] + (size_t)lvl * ne * ne;
          const double *Vp = fVp + (size_t)lvl * mm * mm;
          for (int t = TID; t < ne * ne; t += kThreads) {
            const int a = t / ne, b = t % ne;
            double val = 0.0;
            if (a < m && b < m) val = Vp[a * ne + b];
            else if (b == ne - 1 && a < m) val = fv[(size_t)lvl * mm + a];
            else if (a == ne - 1 && b == ne - 1) val = frho[lvl];
            V[t] = val;
          }
          SYNC();
        }
        const double is = 1.0 / sch;
        double *Mi = w.Minv[sp];
        for (int t = TID; t < ne * ne; t += kThreads) {
          const int a = t / ne, b = t % ne;
          double val;
          if (a < m && b < m) val = Mred[a * m + b] + is * acol[a] * brow[b];
          else if (a < m) val = -is * acol[a];
          else if (b < m) val = -is * brow[b];
          else val = is;
          Mi[t] = val;
        }
        int *nocc = L.iscal + 64;
        for (int a = TID; a < m; a += kThreads) nocc[a] = occ[perm_col(a, k, ne)];
        SYNC();
        for (int a = TID; a < m; a += kThreads) w.occ[sp][a] = nocc[a];
        if (TID == 0) {
          w.occ[sp][ne - 1] = j;
          w.sc->fock_logw[sp] += lr;
          w.sc->fock_sign[sp] *= (int)sr;
        }
      }
    }
  }
  SYNC();
  if (ratio_out && TID == 0) *ratio_out = ratio;
  return accepted;
}

// index of the nth empty site (ascending) of spin sp
__device__ int nth_empty(const WalkerDesc &w, int sp, int nth, Lds &L) {
  const int N = w.N, ne = w.ne[sp];
  int *const fmark = w.fmark + (size_t)sp * N;
  for (int i = TID; i < N; i += kThreads) fmark[i] = 0;
  SYNC();
  for (int a = TID; a < ne; a += kThreads) fmark[w.occ[sp][a]] = 1;
  SYNC();
  const int chunk = (N + kThreads - 1) / kThreads;
  int cnt = 0;
  for (int i = TID * chunk; i < min(N, (TID + 1) * chunk); ++i) cnt += fmark[i] == 0;
  int *counts = L.iscal + 64;
  counts[TID] = cnt;
  SYNC();
  if (TID == 0) {
    int acc = 0, owner = 0;
    for (int t = 0; t < kThreads; ++t) {
      if (acc + counts[t] > nth) { owner = t; break; }
      acc += counts[t];
    }
    int site = -1, c = acc;
    for (int i = owner * chunk; i < min(N, (owner + 1) * chunk); ++i)
      if (fmark[i] == 0) {
        if (c == nth) { site = i; break; }
        ++c;
      }
    L.iscal[3] = site;
  }
  SYNC();
  const int s = L.iscal[3];
  SYNC();
  return s;
}

// One workgroup per (walker, spin): the two species have separate stacks,
// inverses and occupations, so their swap sequences are independent.
// LEAN as for k_left_stack.
template <typename F, bool LEAN>
__global__ void __launch_bounds__(kThreads) k_fock(const WalkerDesc *__restrict__ descs, LdsPlan pl) {
  const WalkerDesc &w = descs[blockIdx.x >> 1];
  const int sp = blockIdx.x & 1;
  Lds L = carve<LEAN>(pl);
  if constexpr (!LEAN) bind_mats(L, w, pl, sp);
  load_bonds(w, L, pl.bond_words);
  // column storage: LDS when the plan holds N entries of F, else device memory
  F *fw = (L.phi && (size_t)pl.phi_elems * sizeof(double) >= (size_t)w.N * sizeof(F))
              ? reinterpret_cast<F *>(L.phi)
              : reinterpret_cast<F *>(w.fw + (size_t)sp * w.N);
  const uint32_t sweep = (uint32_t)w.sc->sweep;
  const int ne = w.ne[sp];
  if ((w.flags & 1) || ne == 0 || ne == w.N) return;
  for (int t = 0; t < ne; ++t) {
    const int k = pick(uniform01(w.seed, w.wid, kSwapK, sweep, (uint32_t)sp, (uint32_t)t), ne);
    const int jn = pick(uniform01(w.seed, w.wid, kSwapJ, sweep, (uint32_t)sp, (uint32_t)t), w.N - ne);
    const int j = nth_empty(w, sp, jn, L);
    const double xacc = uniform01(w.seed, w.wid, kSwapAcc, sweep, (uint32_t)sp, (uint32_t)t);
    double rr = 0.0;
    const bool acc = j >= 0 && swap_move(w, sp, k, j, xacc, true, L, fw, &rr);
    if (TID == 0) {
      w.sc->swap_att[sp] += 1;
      if (acc) w.sc->swap_acc[sp] += 1;
      if (rr != 0.0) w.sc->swap_near[sp] += near_tie_lane(xacc, fabs(rr));
    }
    SYNC();
  }
}

// ---------------------------------------------------------------------------
// Parity surface
// ---------------------------------------------------------------------------
// stabilised right state B_b ... B_1 P (QR at multiples of n_stab and at b) in PhiR
__device__ void right_state(const WalkerDesc &w, int sp, int b, Lds &L) {
  const int m = w.ne[sp];
  double *Phi = w.PhiR[sp];
  fill_P(w, sp, Phi);
  for (int l = 1; l <= b; ++l) {
    apply_diag(w, Phi, m, l, sp, false);
    apply_ek(w, L, Phi, m);
    if (l % w.nstab == 0 || l == b) cholqr<double>(Phi, w.T[sp], Phi, nullptr, nullptr, w.fVp, w.N, m, L, w.sc);
  }
}
// stabilised left state (P^T B_L ... B_{b+1})^T in X
__device__ void left_state(const WalkerDesc &w, int sp, int b, Lds &L) {
  const int m = w.ne[sp];
  double *Y = w.X[sp];
  fill_P(w, sp, Y);
  int cnt = 0;
  for (int l = w.L; l > b; --l) {
    apply_ekT(w, L, Y, m);
    apply_diag(w, Y, m, l, sp, false);
    if (++cnt % w.nstab == 0 || l == b + 1) cholqr<double>(Y, w.T[sp], Y, nullptr, nullptr, w.fVp, w.N, m, L, w.sc);
  }
}

__global__ void __launch_bounds__(kThreads) k_green(const WalkerDesc *__restrict__ descs, int mm, int b, int sp, double *G) {
  const WalkerDesc &w = descs[0];
  const LdsPlan pl = parity_plan(mm);
  Lds L = carve(pl);
  bind_mats(L, w, pl, 0);
  const int N = w.N, m = w.ne[sp];
  right_state(w, sp, b, L);
  left_state(w, sp, b, L);
  gram(w.X[sp], m, w.PhiR[sp], m, N, L.A, L.red);
  double la;
  int sg;
  if (m > 0) gj_inverse(L.A, L.B, m, L, &la, &sg);
  // T = Phi_R M^{-1}
  for (int t = TID; t < N * m; t += kThreads) {
    const int i = t / m, c = t % m;
    double s = 0.0;
    for (int a = 0; a < m; ++a) s += w.PhiR[sp][(size_t)i * m + a] * L.B[a * m + c];
    w.T[sp][t] = s;
  }
  SYNC();
  for (size_t t = TID; t < (size_t)N * N; t += kThreads) {
    const int i = (int)(t / N), jj = (int)(t % N);
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += w.T[sp][(size_t)i * m + c] * w.X[sp][(size_t)jj * m + c];
    G[t] = (i == jj ? 1.0 : 0.0) - s;
  }
}

__global__ void __launch_bounds__(kThreads) k_flip_ratio(const WalkerDesc *__restrict__ descs, int mm, int slice, int site) {
  const WalkerDesc &w = descs[0];
  const LdsPlan pl = parity_plan(mm);
  Lds L = carve(pl);
  bind_mats(L, w, pl, 0);
  const int N = w.N, l = slice + 1;
  double r = 1.0;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    if (m == 0) continue;
    right_state(w, sp, l - 1, L);
    apply_diag(w, w.PhiR[sp], m, l, sp, false);
    left_state(w, sp, l, L);
    apply_ekT(w, L, w.X[sp], m);
    gram(w.X[sp], m, w.PhiR[sp], m, N, L.A, L.red);
    double la;
    int sg;
    gj_inverse(L.A, L.B, m, L, &la, &sg);
    double a = 0.0;
    if (TID == 0) {
      for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q)
          a += w.PhiR[sp][(size_t)site * m + p] * L.B[p * m + q] * w.X[sp][(size_t)site * m + q];
      const int ss = (sp == 0 ? 1 : -1) * w.s[(size_t)slice * N + site];
      const double delta = ss > 0 ? w.delta_dn_s : w.delta_up_s;
      r *= 1.0 + delta * a;
    }
    SYNC();
  }
  if (TID == 0) w.dbg[0] = r;
}

__global__ void __launch_bounds__(kThreads) k_swap_ratio(const WalkerDesc *__restrict__ descs, int mm, int sp, int k, int j) {
  const WalkerDesc &w = descs[0];
  const LdsPlan pl = parity_plan(mm);
  Lds L = carve(pl);
  bind_mats(L, w, pl, 0);
  for (int s2 = 0; s2 < 2; ++s2) {
    right_stack(w, s2, L, w.PhiR[s2]);
    double la;
    int sg;
    inverse_at_beta(w, s2, L, &la, &sg);
  }
  swap_move(w, sp, k, j, 2.0, false, L, w.fw, w.dbg);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int clamp_mm(int mm) { return mm < 1 ? 1 : mm; }

// allow dynamic LDS above the 64 KiB default

// ---------------------------------------------------------------------------
// Constrained-path (phaseless) inner walk of one Fock state eta (SM Sec. VI).
// Each random walker propagates Phi = P_eta through B_l(s) = E_K D0 F_l(s),
// drawing its Ising fields site by site against the backward trial state of
// the one-body Hamiltonian, X_l = (B0_L ... B0_{l+1} E_K)^T P_eta: the left
// stack of the U = 0 trial walker, stored at every slice's flip point.  The
// overlap matrix X_l^T Phi does not change across E_K D0 (the trial state
// moves back by the same factor), so the inverse carries over from slice to
// slice and each site's ratio is the rank-1 one,
//   r_sigma(s) = 1 + (e^{sigma lambda s} - 1) g_sigma,
//   g_sigma = Phi[i,:] (X^T Phi)^{-1} X[i,:]^T,
// followed by the Sherman-Morrison update of the inverse and the row scaling
// Phi[i,:] *= e^{sigma lambda s} (two barriers per site: every wave takes the
// decision itself from the same values).  Phaseless cut: a factor max(0, r); a
// walker whose factor is 0 is dead and draws nothing more.  Field draws:
//   importance: p(+1) = max(0, r(+1)) / (max(0, r(+1)) + max(0, r(-1))),
//               weight times (max(0, r(+1)) + max(0, r(-1))) / 2;
//   free:       p(+1) = 1/2, weight times max(0, r(s)).
// Walkers are QR'd at block ends (Phi -> Q; the scale cancels in every
// ratio) and their inverse is formed afresh at block starts.
// One workgroup per walker, inverses in LDS (Ne <= 64 per spin); the rows of
// the next site are loaded while the current site's update runs.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_cp_init(const WalkerDesc *__restrict__ trial, CpDesc cp) {
  const WalkerDesc &w = *trial;
  const int a = blockIdx.x, N = w.N;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    double *ph = cp.cur.phi[sp] + (size_t)a * N * m;
    for (size_t t = TID; t < (size_t)N * m; t += kThreads) ph[t] = 0.0;
    __syncthreads();
    for (int q = TID; q < m; q += kThreads) ph[(size_t)w.occ[sp][q] * m + q] = 1.0;
  }
  int8_t *path = cp.cur.s + (size_t)a * w.L * N;
  for (size_t t = TID; t < (size_t)w.L * N; t += kThreads) path[t] = 0;
  if (TID == 0) {
    cp.cur.logw[a] = 0.0;
    cp.cur.logq[a] = 0.0;
    cp.cuts[a] = 0;
  }
}

__global__ void __launch_bounds__(kThreads) k_cp_walk(const WalkerDesc *__restrict__ trial, CpDesc cp, LdsPlan pl,
                                                      int l_begin, int l_end, uint32_t tag) {
  const WalkerDesc &w = *trial;
  const int a = blockIdx.x, N = w.N;
  Lds L = carve(pl);
  load_bonds(w, L, pl.bond_words);
  if (cp.cur.logw[a] == -INFINITY) return;   // dead: the same value for every thread
  const int ne[2] = {w.ne[0], w.ne[1]};
  double *phi[2], *Ms[2] = {L.Ms0, L.Ms1};
  for (int sp = 0; sp < 2; ++sp) phi[sp] = cp.cur.phi[sp] + (size_t)a * N * ne[sp];
  int8_t *path = cp.cur.s + (size_t)a * w.L * N;
  double *rows = L.vec;       // [2 buf][x0, p0, x1, p1][64]: rows of the current and the next site
  double *uv = L.uw;          // [u0, v0, u1, v1][64]
  // a segment that starts inside a block resumes with the stored inverse
  if ((l_begin - 1) % w.nstab != 0)
    for (int sp = 0; sp < 2; ++sp)
      for (int t = TID; t < ne[sp] * ne[sp]; t += kThreads)
        Ms[sp][t] = cp.cur.minv[sp][(size_t)a * ne[sp] * ne[sp] + t];
  double logw = cp.cur.logw[a], logq = cp.cur.logq[a];   // thread 0's running sums
  __syncthreads();
  const int grp = TID >> 6, t = TID & 63, gsp = grp >> 1;
  bool dead = false;
  for (int l = l_begin; l <= l_end && !dead; ++l) {
    const int k = (l - 1) / w.nstab + 1;
    const int l0 = (k - 1) * w.nstab + 1, l1 = min(k * w.nstab, w.L);
    const double *X[2];
    for (int sp = 0; sp < 2; ++sp) {
      X[sp] = w.LX[sp] + (size_t)(l - 1) * N * ne[sp];
      apply_diag(w, phi[sp], ne[sp], l, sp, false);   // D0: the trial walker's lambda is 0
    }
    if (l == l0)
      for (int sp = 0; sp < 2; ++sp) {
        if (ne[sp] == 0) continue;
        gram(X[sp], ne[sp], phi[sp], ne[sp], N, L.A, L.red);
        double la;
        int sg;
        gj_inverse(L.A, Ms[sp], ne[sp], L, &la, &sg);
      }
    // rows of site 0: group grp (x0, p0, x1, p1) loads its row
    {
      const int m = ne[gsp];
      const double *src = (grp & 1) ? phi[gsp] : X[gsp];
      if (t < m) rows[grp * 64 + t] = src[t];
    }
    __syncthreads();
    for (int i = 0; i < N; ++i) {
      const double *rb = rows + (i & 1) * 256;
      double *rn = rows + ((i + 1) & 1) * 256;
      // u = M^{-1} x and v = p M^{-1}, one entry per thread
      {
        const int m = ne[gsp];
        const double *M = Ms[gsp];
        if (t < m) {
          double acc = 0.0;
          if ((grp & 1) == 0) {
            const double *x = rb + gsp * 128;
            for (int q = 0; q < m; ++q) acc += M[t * m + q] * x[q];
          } else {
            const double *pr = rb + gsp * 128 + 64;
            for (int q = 0; q < m; ++q) acc += pr[q] * M[q * m + t];
          }
          uv[grp * 64 + t] = acc;
        }
      }
      __syncthreads();
      // every wave forms g and takes the decision from the same LDS values in
      // the same order, so every thread holds the same result and no barrier
      // is needed before the update
      double c0 = 0.0, c1 = 0.0, f0 = 1.0, f1 = 1.0;
      {
        double g0 = t < ne[0] ? rb[64 + t] * uv[t] : 0.0;
        double g1 = t < ne[1] ? rb[192 + t] * uv[128 + t] : 0.0;
        g0 = wave_sum_d(g0);
        g1 = wave_sum_d(g1);
        double f[2];
        for (int u = 0; u < 2; ++u) {
          const double r = (1.0 + cp.delta[0][u] * g0) * (1.0 + cp.delta[1][u] * g1);
          f[u] = r > 0.0 ? r : 0.0;
        }
        const double x = uniform01(cp.seed, (uint64_t)a, kCpField, tag, (uint32_t)(l - 1), (uint32_t)i);
        int u = 0;
        double factor = 0.0, pq = 1.0;
        if (cp.mode == 0) {
          const double Ni = 0.5 * f[0] + 0.5 * f[1];
          if (Ni != 0.0) {
            const double pp = 0.5 * f[0] / Ni;
            u = x < pp ? 0 : 1;
            factor = Ni;
            pq = u == 0 ? pp : 1.0 - pp;
          }
        } else {
          u = x < 0.5 ? 0 : 1;
          factor = f[u];
        }
        if (factor == 0.0) {
          dead = true;
          if (TID == 0) logw = -INFINITY;
        } else {
          if (TID == 0) {
            logw += log(factor);
            if (cp.mode == 0) logq += log(pq);
            path[(size_t)(l - 1) * N + i] = (int8_t)(u == 0 ? 1 : -1);
          }
          const double d0 = cp.delta[0][u], d1 = cp.delta[1][u];
          c0 = d0 / (1.0 + d0 * g0);
          c1 = d1 / (1.0 + d1 * g1);
          f0 = 1.0 + d0;
          f1 = 1.0 + d1;
        }
      }
      if (dead) break;
      // the next site's rows (its p row is not touched by this update)
      if (i + 1 < N) {
        const int m = ne[gsp];
        const double *src = (grp & 1) ? phi[gsp] : X[gsp];
        if (t < m) rn[grp * 64 + t] = src[(size_t)(i + 1) * m + t];
      }
      for (int sp = 0; sp < 2; ++sp) {
        const int m = ne[sp];
        const double c = sp == 0 ? c0 : c1;
        const double *u = uv + sp * 128, *v = uv + sp * 128 + 64;
        for (int e = TID; e < m * m; e += kThreads) {
          const int p = e / m, q = e - p * m;
          Ms[sp][e] -= c * u[p] * v[q];
        }
        if (TID < m) phi[sp][(size_t)i * m + TID] *= sp == 0 ? f0 : f1;
      }
      __syncthreads();
    }
    if (dead) break;
    for (int sp = 0; sp < 2; ++sp) apply_ek(w, L, phi[sp], ne[sp]);
    if (l == l1)
      for (int sp = 0; sp < 2; ++sp) {
        const int m = ne[sp];
        if (m == 0) continue;
        cholqr<double>(phi[sp], cp.tmp[sp] + (size_t)a * N * m, phi[sp], nullptr, nullptr,
                       cp.vacc + ((size_t)a * 2 + sp) * cp.mm * cp.mm, N, m, L, w.sc);
      }
  }
  __syncthreads();
  if (!dead)
    for (int sp = 0; sp < 2; ++sp)
      for (int e = TID; e < ne[sp] * ne[sp]; e += kThreads)
        cp.cur.minv[sp][(size_t)a * ne[sp] * ne[sp] + e] = Ms[sp][e];
  if (TID == 0) {
    cp.cur.logw[a] = logw;
    cp.cur.logq[a] = logq;
    if (dead) cp.cuts[a] += 1;
  }
}

// comb over the cumulative weights (one thread, in walker order): copy j
// takes the walker whose interval holds (j + xi) W / nw (the nearest live
// walker if rounding lands on a dead one's empty interval); log_pc gains the
// log of the mean weight
__global__ void __launch_bounds__(64) k_cp_comb(CpDesc cp, int l, uint32_t tag) {
  if (threadIdx.x != 0) return;
  const int nw = cp.nw;
  double mx = -INFINITY;
  for (int a = 0; a < nw; ++a) mx = fmax(mx, cp.cur.logw[a]);
  if (mx == -INFINITY) {
    for (int j = 0; j < nw; ++j) cp.pick[j] = -1;
    return;
  }
  double W = 0.0;
  for (int a = 0; a < nw; ++a) W += exp(cp.cur.logw[a] - mx);
  const double xi = uniform01(cp.seed, 0, kCpComb, tag, (uint32_t)(l - 1), 0);
  int a = 0;
  double cum = exp(cp.cur.logw[0] - mx);
  for (int j = 0; j < nw; ++j) {
    const double tpos = ((double)j + xi) * W / (double)nw;
    while (a < nw - 1 && cum <= tpos) {
      ++a;
      cum += exp(cp.cur.logw[a] - mx);
    }
    int b = a;
    while (b > 0 && cp.cur.logw[b] == -INFINITY) --b;
    while (b < nw - 1 && cp.cur.logw[b] == -INFINITY) ++b;
    cp.pick[j] = b;
  }
  cp.log_pc[0] += mx + log(W / (double)nw);
}

// copy j of the comb: the state of walker pick[j] into slot j of dst, weight 1
__global__ void __launch_bounds__(kThreads) k_cp_copy(const WalkerDesc *__restrict__ trial, CpDesc cp, CpState dst) {
  const WalkerDesc &w = *trial;
  const int j = blockIdx.x, src = cp.pick[j] < 0 ? j : cp.pick[j];
  const int N = w.N;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = w.ne[sp];
    const double *ps = cp.cur.phi[sp] + (size_t)src * N * m;
    double *pd = dst.phi[sp] + (size_t)j * N * m;
    for (size_t t = TID; t < (size_t)N * m; t += kThreads) pd[t] = ps[t];
    const double *ms = cp.cur.minv[sp] + (size_t)src * m * m;
    double *md = dst.minv[sp] + (size_t)j * m * m;
    for (int t = TID; t < m * m; t += kThreads) md[t] = ms[t];
  }
  const int8_t *ss = cp.cur.s + (size_t)src * w.L * N;
  int8_t *sd = dst.s + (size_t)j * w.L * N;
  for (size_t t = TID; t < (size_t)w.L * N; t += kThreads) sd[t] = ss[t];
  if (TID == 0) {
    // every walker dead (pick < 0): the population is carried over as it is
    dst.logw[j] = cp.pick[j] < 0 ? cp.cur.logw[j] : 0.0;
    dst.logq[j] = cp.cur.logq[src];
  }
}

// The dynamic-LDS limit of a kernel is raised once to the largest size asked
// for; later launches (also those recorded into a graph) make no call.
template <typename K>
static void lds_attr(K kernel, size_t bytes) {
  if (bytes <= 65536) return;
  static std::mutex mu;   // contexts may be driven from different host threads
  std::lock_guard<std::mutex> guard(mu);
  static const void *keys[64];
  static size_t done[64];
  const void *k = (const void *)kernel;
  int slot = -1;
  for (int t = 0; t < 64; ++t)
    if (keys[t] == k || keys[t] == nullptr) { slot = t; break; }
  if (slot >= 0 && keys[slot] == k && done[slot] >= bytes) return;
  (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (slot >= 0) { keys[slot] = k; done[slot] = bytes > done[slot] ? bytes : done[slot]; }
}

hipError_t launch_init(const WalkerDesc *d, int draw_fields, int draw_occ, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(kThreads), 0, st, d, draw_fields, draw_occ);
  return hipGetLastError();
}
static LdsPlan clamp_plan(LdsPlan p) {
  p.mm = clamp_mm(p.mm);
  return p;
}
hipError_t launch_cp_init(const WalkerDesc *trial, CpDesc cp, hipStream_t st) {
  hipLaunchKernelGGL(k_cp_init, dim3(cp.nw), dim3(kThreads), 0, st, trial, cp);
  return hipGetLastError();
}
hipError_t launch_cp_walk(const WalkerDesc *trial, CpDesc cp, LdsPlan p, int l_begin, int l_end, uint32_t tag,
                          hipStream_t st) {
  p = clamp_plan(p);
  const size_t b = lds_bytes(p);
  lds_attr(k_cp_walk, b);
  hipLaunchKernelGGL(k_cp_walk, dim3(cp.nw), dim3(kThreads), b, st, trial, cp, p, l_begin, l_end, tag);
  return hipGetLastError();
}
hipError_t launch_cp_comb(CpDesc cp, CpState dst, const WalkerDesc *trial, int l, uint32_t tag, hipStream_t st) {
  hipLaunchKernelGGL(k_cp_comb, dim3(1), dim3(64), 0, st, cp, l, tag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cp_copy, dim3(cp.nw), dim3(kThreads), 0, st, trial, cp, dst);
  return hipGetLastError();
}
hipError_t launch_fresh_weight(const WalkerDesc *d, int n, LdsPlan p, int set_tracked, hipStream_t st) {
  p = clamp_plan(p);
  const size_t b = lds_bytes(p);
  lds_attr(k_fresh_weight, b);
  hipLaunchKernelGGL(k_fresh_weight, dim3(n), dim3(kThreads), b, st, d, p, set_tracked);
  return hipGetLastError();
}
// the lean kernels of the per-spin phases: every work matrix in LDS, no
// delayed-chain area, vectors of 64
static bool lean_plan(const LdsPlan &p) { return p.gm == 0 && p.dgn == 0 && p.mm <= 64; }
template <typename F, bool LEAN>
static void launch_left_t(const WalkerDesc *d, int n, const LdsPlan &p, size_t b, hipStream_t st) {
  lds_attr(k_left_stack<F, LEAN>, b);
  hipLaunchKernelGGL((k_left_stack<F, LEAN>), dim3(2 * n), dim3(kThreads), b, st, d, p);
}
hipError_t launch_left_stack(const WalkerDesc *d, int n, LdsPlan p, int mixed, hipStream_t st) {
  p = clamp_plan(p);
  const size_t b = lds_bytes(p);
  const bool lean = lean_plan(p);
  if (mixed) {
    if (lean) launch_left_t<float, true>(d, n, p, b, st);
    else launch_left_t<float, false>(d, n, p, b, st);
  } else {
    if (lean) launch_left_t<double, true>(d, n, p, b, st);
    else launch_left_t<double, false>(d, n, p, b, st);
  }
  return hipGetLastError();
}
hipError_t launch_measure(const WalkerDesc *d, int n, int slots, LdsPlan p, hipStream_t st) {
  p = clamp_plan(p);
  const size_t b = lds_bytes(p);
  lds_attr(k_measure, b);
  hipLaunchKernelGGL(k_measure, dim3(n * slots), dim3(kThreads), b, st, d, p, slots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_measure_sum, dim3(n), dim3(kThreads), 0, st, d);
  return hipGetLastError();
}
template <int TSEL>
static hipError_t launch_forward_t(const WalkerDesc *d, int n, LdsPlan p, int want_aw, int mixed, hipStream_t st) {
  const size_t b = lds_bytes(p);
  if (mixed) {
    lds_attr(k_forward<TSEL, float>, b);
    hipLaunchKernelGGL((k_forward<TSEL, float>), dim3(n), dim3(kThreads), b, st, d, p, want_aw);
  } else {
    lds_attr(k_forward<TSEL, double>, b);
    hipLaunchKernelGGL((k_forward<TSEL, double>), dim3(n), dim3(kThreads), b, st, d, p, want_aw);
  }
  return hipGetLastError();
}
hipError_t launch_forward(const WalkerDesc *d, int n, LdsPlan p, int tile, int do_measure, int mixed, hipStream_t st) {
  p = clamp_plan(p);
  // the register-tile kernels assume the lean layout (all work matrices in
  // LDS, no delayed-chain area, vectors of 64)
  if ((tile == 1 || tile == 2 || tile == 4) && !lean_plan(p)) tile = -1;
  switch (tile) {
    case 1: return launch_forward_t<1>(d, n, p, do_measure, mixed, st);
    case 2: return launch_forward_t<2>(d, n, p, do_measure, mixed, st);
    case 4: return launch_forward_t<4>(d, n, p, do_measure, mixed, st);
    case kDelayed: return launch_forward_t<kDelayed>(d, n, p, do_measure, mixed, st);
    case kMfma: return launch_forward_t<kMfma>(d, n, p, do_measure, mixed, st);
    case 0: return launch_forward_t<0>(d, n, p, do_measure, mixed, st);
    default: return launch_forward_t<-1>(d, n, p, do_measure, mixed, st);
  }
}
template <typename F, bool LEAN>
static void launch_fock_t(const WalkerDesc *d, int n, const LdsPlan &p, size_t b, hipStream_t st) {
  lds_attr(k_fock<F, LEAN>, b);
  hipLaunchKernelGGL((k_fock<F, LEAN>), dim3(2 * n), dim3(kThreads), b, st, d, p);
}
hipError_t launch_fock(const WalkerDesc *d, int n, LdsPlan p, int mixed, hipStream_t st) {
  p = clamp_plan(p);
  const size_t b = lds_bytes(p);
  const bool lean = lean_plan(p);
  if (mixed) {
    if (lean) launch_fock_t<float, true>(d, n, p, b, st);
    else launch_fock_t<float, false>(d, n, p, b, st);
  } else {
    if (lean) launch_fock_t<double, true>(d, n, p, b, st);
    else launch_fock_t<double, false>(d, n, p, b, st);
  }
  return hipGetLastError();
}
hipError_t launch_green(const WalkerDesc *d, int mm, int b, int sp, double *G, hipStream_t st) {
  mm = clamp_mm(mm);
  const size_t by = lds_bytes(LdsPlan{mm, 0, 1, 0, 0, 0, mm > kLdsNe ? 1 : 0, 0});
  lds_attr(k_green, by);
  hipLaunchKernelGGL(k_green, dim3(1), dim3(kThreads), by, st, d, mm, b, sp, G);
  return hipGetLastError();
}
hipError_t launch_flip_ratio(const WalkerDesc *d, int mm, int slice, int site, hipStream_t st) {
  mm = clamp_mm(mm);
  const size_t by = lds_bytes(LdsPlan{mm, 0, 1, 0, 0, 0, mm > kLdsNe ? 1 : 0, 0});
  lds_attr(k_flip_ratio, by);
  hipLaunchKernelGGL(k_flip_ratio, dim3(1), dim3(kThreads), by, st, d, mm, slice, site);
  return hipGetLastError();
}
hipError_t launch_swap_ratio(const WalkerDesc *d, int mm, int sp, int k, int j, hipStream_t st) {
  mm = clamp_mm(mm);
  const size_t by = lds_bytes(LdsPlan{mm, 0, 1, 0, 0, 0, mm > kLdsNe ? 1 : 0, 0});
  lds_attr(k_swap_ratio, by);
  hipLaunchKernelGGL(k_swap_ratio, dim3(1), dim3(kThreads), by, st, d, mm, sp, k, j);
  return hipGetLastError();
}

}  // namespace lecqmc
