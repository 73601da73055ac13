// Internal structures shared by the host API (lecqmc_capi.hip) and the
// gfx950 kernels (lecqmc_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lecqmc {

constexpr int kThreads = 256;   // one workgroup (4 wave64) per walker
constexpr int kMaxNe = 64;      // particles per spin held in LDS-resident Ne x Ne blocks

// counter-based generator streams (shared layout with the walker's key)
enum Stream : uint32_t { kFlip = 1, kSwapK = 2, kSwapJ = 3, kSwapAcc = 4, kInitField = 5, kInitOcc = 6 };

// Scalars of one walker that kernels update (device memory).
struct Scalars {
  unsigned long long sweep;     // completed sweeps
  double logw;                  // tracked log|W|
  int sign;                     // tracked sign
  int status;                   // 0 ok, bit 1 = QR shift used, bit 2 = singular inverse
  long long flip_att, flip_acc, swap_att, swap_acc, qr_shifted;
  double max_wrap, logw_drift;
  double fresh_logw;            // written by the fresh-weight kernel
  int fresh_sign;
  int pad;
  double dbg[4];
};

// Device descriptor of one walker (copied to device memory at creation).
struct WalkerDesc {
  int N, L, nstab, nblk, ncol, nbonds, nsub, ncells, flags, nobs;
  int ne[2];
  int mmax;                     // max(ne[0], ne[1], 1): stride of the per-level Fock scratch
  uint64_t seed, wid;
  double elam, emlam;           // exp(+lambda), exp(-lambda)
  double delta_dn_s, delta_up_s;// Delta for sigma*s = +1: exp(-2 lambda) - 1 ; sigma*s = -1: exp(2 lambda) - 1
  double wrap_tol;
  const int *col_start;         // [ncol + 1]
  const int *bi, *bj;           // [nbonds], grouped by colour
  const double *bdiag, *boff;   // cosh(dtau h), -sinh(dtau h)
  const double *bh;             // h
  const double *eps_fac;        // exp(-dtau eps_i)
  const double *eps;            // eps_i
  const int *sub;               // sublattice index
  int8_t *s;                    // [L][N]
  int *occ[2];                  // [N] each (first ne used)
  double *LS[2];                // [(nblk + 1)][N][ne]  left states at block boundaries
  double *LX[2];                // [L][N][ne]  left state at the flip point of every slice
  double *RQ[2];                // [nblk][N][ne]
  double *RV[2];                // [nblk][ne][ne]
  double *Minv[2];              // [ne][ne]
  double *PhiR[2];              // [N][ne]
  double *X[2];                 // [N][ne]  (Phi_L transposed)
  double *T[2];                 // [N][ne]  scratch
  double *Aw[2];                // [N] wrapped diagonal of A at block ends
  double *fq;                   // [nblk][N] new columns of an addition
  double *fw;                   // [N] propagated column
  double *fVp;                  // [nblk][ne_max^2]
  double *fgc, *fgs;            // [nblk][ne_max]
  double *fv;                   // [nblk][ne_max]
  double *frho;                 // [nblk]
  int *fmark;                   // [N] occupancy marks / permutation scratch
  double *obs;                  // [nobs]
  double *dbg;                  // [N*N] parity-surface output (N <= dbg_n) else [8]
  Scalars *sc;
};

// kernel launchers (lecqmc_kernels.hip); descs = device array of descriptors.
// phi_elems > 0 keeps the Slater blocks of each walker resident in LDS.
constexpr size_t kLdsLimit = 163840;
size_t lds_bytes(int max_ne, int phi_elems);
hipError_t launch_init(const WalkerDesc *d_desc, int draw_fields, int draw_occ, hipStream_t st);
hipError_t launch_fresh_weight(const WalkerDesc *d_descs, int n, int max_ne, int phi_elems, int set_tracked, hipStream_t st);
hipError_t launch_left_stack(const WalkerDesc *d_descs, int n, int max_ne, int phi_elems, hipStream_t st);
hipError_t launch_forward(const WalkerDesc *d_descs, int n, int max_ne, int phi_elems, int do_measure, hipStream_t st);
hipError_t launch_fock(const WalkerDesc *d_descs, int n, int max_ne, int phi_elems, hipStream_t st);
hipError_t launch_green(const WalkerDesc *d_desc, int max_ne, int boundary, int spin, double *G, hipStream_t st);
hipError_t launch_flip_ratio(const WalkerDesc *d_desc, int max_ne, int slice, int site, hipStream_t st);
hipError_t launch_swap_ratio(const WalkerDesc *d_desc, int max_ne, int spin, int k, int j, hipStream_t st);

}  // namespace lecqmc
