// Internal structures shared by the host API (lecqmc_capi.hip) and the
// gfx950 kernels (lecqmc_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lecqmc {

constexpr int kThreads = 256;   // one workgroup (4 wave64) per walker
constexpr int kMaxNe = 256;     // particles per spin
constexpr int kLdsNe = 64;      // largest Ne whose Ne x Ne work matrices are kept in LDS
constexpr int kDelayed = 9;     // chain shape code of the delayed (submatrix) flip update
constexpr int kDS = 32;         // sites per chunk at most (accepted-site masks are 32 bits)
constexpr int kMfma = 10;       // chain shape code of the delayed update on the FP64 matrix cores
constexpr int kMS = 16;         // sites per chunk of that chain (one 16-wide matrix-core tile)
// Ne rounded up to whole 16-row tiles
__host__ __device__ inline int ne16(int ne) { return (ne + 15) & ~15; }
constexpr int kMfmaMaxNe = 128; // largest Ne of that chain (its W tiles stay in registers)
// LDS doubles of the matrix-core chain's chunk matrices for one walker: G
// then Z (16 x 16, row stride 17) and two partial G (16 x 16) per spin, then
// U (Ne x 16, row stride 17) per spin when it fits the launch
__host__ __device__ inline int mfma_lds_small() { return 2 * 16 * 17 + 2 * 2 * 256; }
__host__ __device__ inline int mfma_lds_doubles(int ne0, int ne1) {
  return mfma_lds_small() + 17 * (ne16(ne0) + ne16(ne1));
}

// counter-based generator streams (shared layout with the walker's key)
enum Stream : uint32_t { kFlip = 1, kSwapK = 2, kSwapJ = 3, kSwapAcc = 4, kInitField = 5, kInitOcc = 6,
                         kCpField = 7, kCpComb = 8 };

// Scalars of one walker that kernels update (device memory).
struct Scalars {
  unsigned long long sweep;     // completed sweeps
  double logw;                  // tracked log|W| (up to the pending Fock terms below)
  int sign;                     // tracked sign
  int status;                   // 0 ok, bit 1 = QR shift used, bit 2 = singular inverse or QR
                                // breakdown, bit 3 = wrap error of a measuring sweep above wrap_tol
  long long flip_att, flip_acc, qr_shifted;
  long long swap_att[2], swap_acc[2];   // per spin (one Fock workgroup per spin)
  long long near_ties;          // flip decisions with |u - |r|| below the near-tie margin
  long long swap_near[2];       // the same for swaps, per spin
  double fock_logw[2];          // log|r| of accepted swaps per spin, folded in by the next forward pass
  int fock_sign[2];
  double max_wrap, logw_drift;
  double fresh_logw;            // written by the fresh-weight kernel
  int fresh_sign;
  int pad;
  double wrap_sweep;            // largest wrap error of the last measuring sweep
  long long fwd_ticks;          // wall-clock ticks of the last forward pass of this walker
  double dbg[4];
};

// Device descriptor of one walker (copied to device memory at creation).
struct WalkerDesc {
  int N, L, nstab, nblk, ncol, nbonds, nsub, ncells, flags, nobs;
  int mixed;                    // 1: FP32 slice propagation (LECQMC_MIXED)
  int ne[2];
  int mmax;                     // max(ne[0], ne[1], 1): stride of the per-level Fock scratch
  // shape of the flip chain (set by the host: default by Ne, or autotuned)
  int tile;                     // register tile T (Ne <= 8T held in registers), 0 (inverse in LDS),
                                // kDelayed or kMfma (delayed chunk updates)
  int chunk;                    // sites per staged chunk, 4..32
  int xld;                      // row stride of the staged rows: 8T, or mmax when tile = 0
  uint64_t seed, wid;
  double elam, emlam;           // exp(+lambda), exp(-lambda)
  double delta_dn_s, delta_up_s;// Delta for sigma*s = +1: exp(-2 lambda) - 1 ; sigma*s = -1: exp(2 lambda) - 1
  double wrap_tol;
  const int *col_start;         // [ncol + 1]
  const int *bi, *bj;           // [nbonds], grouped by colour
  const double *bdiag, *boff;   // cosh(dtau h), -sinh(dtau h)
  const double *bh;             // h
  // compact copy for LDS: i | j << 16, index of (cosh, -sinh) in coef
  const int *bij;               // [nbonds]
  const uint8_t *bci;           // [nbonds]
  const double *coef;           // [ncoef][2]
  int ncoef;                    // distinct bond coefficients (0 = no compact copy)
  int bond_words;               // 4-byte words of the compact copy in LDS
  const double *eps_fac;        // exp(-dtau eps_i)
  const double *eps;            // eps_i
  const int *sub;               // sublattice index
  int8_t *s;                    // [L][N]
  int *occ[2];                  // [N] each (first ne used)
  double *LS[2];                // [(nblk + 1)][N][ne]  left states at block boundaries
  double *LX[2];                // [L][N][ne]  left state at the flip point of every slice
                                // (FP32 entries for mixed-precision walkers)
  double *RQ[2];                // [nblk][N][ne]
  double *RV[2];                // [nblk][ne][ne]
  double *Minv[2];              // [ne][ne]
  double *PhiR[2];              // [N][ne]
  double *X[2];                 // [N][ne]  (Phi_L transposed)
  double *T[2];                 // [N][ne]  scratch
  double *Aw[2];                // [nblk][N] diagonal of A from the carried inverse at block ends
  double *mpart;                // [slots][nobs + 1] per-boundary measurement records
  double *mscr;                 // [slots][mscr_stride] measurement scratch
  size_t mscr_stride;
  // Fock-phase scratch, [2 spins] x ...; fVp spin 0 also serves as QR scratch
  double *fq;                   // [2][nblk][N] new columns of an addition
  double *fw;                   // [2][N] propagated column
  double *fVp;                  // [2][nblk][mmax^2]
  double *fgc, *fgs;            // [2][nblk][mmax]
  double *fv;                   // [2][nblk][mmax]
  double *frho;                 // [2][nblk]
  int *fmark;                   // [2][N] occupancy marks / permutation scratch
  double *obs;                  // [nobs]
  double *dbg;                  // [N*N] parity-surface output (N <= dbg_n) else [8]
  double *dch;                  // delayed flip chain: [2 spins][U, W, U~, W~: mmax x kDS each] +
                                // [2 (row, column)][2 spins][kDS][kDS] records
  double *bigm;                 // [2 slots][4][mmax^2] the Ne x Ne work matrices of a launch whose
                                // largest Ne exceeds kLdsNe (slot = spin in per-spin kernels)
  Scalars *sc;
};

// LDS plan of one launch: the largest Ne (mm; the Ne x Ne work matrices move
// to device memory in part or whole when they do not fit, gm), the room for resident Slater
// blocks (phi_elems doubles; a walker whose blocks fit keeps them there, the
// others stream them), right-row staging buffers (forward pass with a
// streamed walker), the compact bond tables (bond_words, 0 = read from device
// memory) and the flip-chain staging area (xs_elems doubles for the largest
// 4 * chunk * xld of the launch, smax = its largest chunk; 0 outside the
// forward pass).
struct LdsPlan {
  int mm, phi_elems, stage_ps, bond_words, xs_elems, smax;
  int gm;   // Ne x Ne work matrices: 0 all four in LDS, 2 the inverses in LDS and the scratch
            // pair in each walker's bigm, 1 all four in bigm
  int dgn;  // LDS doubles for the delayed chains' chunk and coefficient matrices (4 kDS^2 for
            // kDelayed, mfma_lds_doubles for kMfma, or 0)
};
// LDS doubles that a walker's resident blocks of `entries` elements need
__host__ __device__ inline long phi_doubles(long entries, int elem_bytes) {
  return (entries * elem_bytes + 7) / 8;
}
constexpr size_t kLdsLimit = 163840;
constexpr int kMaxCoef = 16;
size_t lds_bytes(const LdsPlan &p);
// kernel launchers (lecqmc_kernels.hip); descs = device array of descriptors.
hipError_t launch_init(const WalkerDesc *d_desc, int draw_fields, int draw_occ, hipStream_t st);
hipError_t launch_fresh_weight(const WalkerDesc *d_descs, int n, LdsPlan p, int set_tracked, hipStream_t st);
// mixed != 0: FP32 storage and propagation of the Slater blocks, stored left
// states and Fock columns (every walker of the launch must be mixed)
hipError_t launch_left_stack(const WalkerDesc *d_descs, int n, LdsPlan p, int mixed, hipStream_t st);
// tile: the chain shape shared by every walker of the launch (1, 2, 4 or 0),
// or -1 when they differ (each walker's own shape is dispatched in the kernel)
hipError_t launch_forward(const WalkerDesc *d_descs, int n, LdsPlan p, int tile, int do_measure, int mixed,
                          hipStream_t st);
hipError_t launch_fock(const WalkerDesc *d_descs, int n, LdsPlan p, int mixed, hipStream_t st);
hipError_t launch_measure(const WalkerDesc *d_descs, int n, int slots, LdsPlan p, hipStream_t st);
hipError_t launch_green(const WalkerDesc *d_desc, int max_ne, int boundary, int spin, double *G, hipStream_t st);
hipError_t launch_flip_ratio(const WalkerDesc *d_desc, int max_ne, int slice, int site, hipStream_t st);
hipError_t launch_swap_ratio(const WalkerDesc *d_desc, int max_ne, int spin, int k, int j, hipStream_t st);

// Constrained-path population of one Fock state (device arrays, one set of
// walker states; the comb copies into a second set).  The trial walker (U = 0,
// the same Fock state) supplies the tables and, from its left stack, the
// backward trial states at every slice.
struct CpState {
  double *phi[2];       // [nw][N][ne]   walker Slater blocks
  double *minv[2];      // [nw][ne][ne]  (X^T Phi)^{-1} at a segment end
  int8_t *s;            // [nw][L][N]    drawn field path
  double *logw, *logq;  // [nw]
};
struct CpDesc {
  CpState cur;
  double *tmp[2];       // [nw][N][ne]   QR scratch
  double *vacc;         // [nw][2][mm][mm] QR scratch
  long long *cuts;      // [nw]
  int *pick;            // [nw] comb sources
  double *log_pc;       // [1] sum of log(mean weight) over the combs
  int nw, mode, mm;
  uint64_t seed;
  double delta[2][2];   // [spin][s = +1, -1]: exp(sigma lambda s) - 1
};
hipError_t launch_cp_init(const WalkerDesc *trial, CpDesc cp, hipStream_t st);
hipError_t launch_cp_walk(const WalkerDesc *trial, CpDesc cp, LdsPlan p, int l_begin, int l_end, uint32_t tag,
                          hipStream_t st);
// comb after slice l: sources from cp.cur's weights, states copied into dst
hipError_t launch_cp_comb(CpDesc cp, CpState dst, const WalkerDesc *trial, int l, uint32_t tag, hipStream_t st);

}  // namespace lecqmc
