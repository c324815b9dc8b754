// Internal declarations of libpolyaipm: handle layout, device descriptors of
// a batch, and launch wrappers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "polyaipm.h"

namespace psdp {

constexpr int kMaxN = 128;   // largest block order held whole in LDS (128 KB)
constexpr int kTB = 8;       // index-group size of the tiled basis
constexpr int kNB = 64;      // Schur Cholesky tile
constexpr int kPairGrid = 1024;   // workgroups of the whole-pair assembly (grid-stride)
constexpr int kBwdCW = 16;   // columns of a backward-sweep workgroup's strip (divides 64)
constexpr int kSW = 8;       // default Cholesky panels per super-panel (depth of the wide update / 64)
// 64 x 64 output tiles of an n x n block (the workgroups a block product
// takes when its tiles are shared out over a grid's y dimension)
inline int gemm_tiles(int n) { return ((n + 63) / 64) * ((n + 63) / 64); }
constexpr int kLeftMaxP = 64;  // the autotuner tries the left-looking factorisation below this many tiles
constexpr int kMaxDeg = 20;  // largest multinomial degree (20! < 2^63)
constexpr int kNSC = 32;     // per-system scalar slots

// per-system scalar slots (double array sc[sys * kNSC + slot])
enum Slot {
  S_PHI = 0, S_PSI, S_TRZX, S_PINF, S_DINF, S_GAPABS, S_GAPREL, S_MU, S_TP, S_TD,
  S_NORMBX, S_ONE, S_MINUS_ONE, S_TLAST, S_STT, S_NORMC, S_NORMA, S_DIAGMAX, S_TAU,
  S_IRETA,   // largest ||rhs - Lambda x0|| / ||rhs|| of the iteration's refined solves
  S_IRLAST,  // residual ratio of the latest refinement step
  S_IRFAIL,  // 1 if a solve of the iteration stopped refining above kIrAccept
  S_IRSTEPS, // refinement corrections applied in the iteration
  S_TPA, S_TDA,   // step lengths of the predictor directions (Mehrotra's sigma), -1: none
  S_MUDELTA,      // change of mu made by Mehrotra's sigma
};

// per-system flag bits (int array flags[sys])
enum Flag {
  F_ACTIVE = 1,       // takes part in the current iteration
  F_ZFAIL = 2,        // a block of Z failed Cholesky
  F_LAMFAIL = 4,      // the Schur matrix failed Cholesky
  F_LADDERFAIL = 8,   // the step ladder ran out
  F_CHOLSEL = 16,     // selected for the (re)factorisation pass
  F_ASM32 = 32,       // Schur assembly in reduced precision this iteration
  F_PARK = 64,        // temporarily inactive (FP64-assembled system during refinement)
  F_SHIFTED = 128,    // the Schur matrix is factored with a diagonal shift this step
};

// Failure policy of the FP64 Schur factorisation: the step is retried on
// Lambda + f max_i Lambda_ii I, f = kShiftFirst, then x kShiftGrowth per
// failure up to the caller's limit, and its solves are refined against the
// unshifted matrix-free product with at most kIrShift corrections (more if
// ir_max asks for more).
constexpr double kShiftFirst = 1e-14;
constexpr double kShiftGrowth = 100.0;
constexpr int kIrShift = 6;

// Iterative refinement of the Newton solves: a solve is accepted once its
// residual ratio ||rhs - Lambda x||_inf / ||rhs||_inf falls to kIrTol, or
// stops falling (by half per step) at or below kIrAccept.  A system whose
// solve is not accepted, whose first ratio exceeds kIrSwitch, or whose
// reduced-precision Schur matrix fails Cholesky is assembled in FP64 from
// the next iteration on.
constexpr double kIrTol = 1e-14;
constexpr double kIrAccept = 1e-10;
constexpr double kIrSwitch = 1e-1;

struct SysDesc {
  int n, L0, L, M, Nt, nb, P, mode;   // P = Kpad / kNB; mode 0 paper SDP, 1 phase-I
  // n is the order of every block; the basis matrices are nbas x nbas, placed
  // on the diagonal copies times (discrete form: n = 2 nbas, copies = 2)
  int nbas, copies;
  int K, Kpad, blk0, npairs_hm;
  int sw, ssw;      // Schur Cholesky: panels per super-panel (wide update depth 64 sw) and
                    // per sub-panel inside it (its update depth 64 ssw; ssw = sw: none)
  int64_t boff;     // block arena offset (doubles) of the system's first block
  int64_t voff;     // vector offset (Kpad entries per vector)
  int64_t loff;     // Schur matrix offset (Kpad * Kpad)
  int64_t poff;     // P_h scratch offset (L0 * n * n)
  int64_t dgoff;    // factored diagonal tiles of the Schur matrix (P * 64 * 64)
  int64_t pboff;    // panel buffer of the fused factorisation (2 P 64^2), -1: none
  int64_t gioff;    // grouped solves: inverses of the factor's diagonal blocks of
                    // kSG tiles, (L_qq^-1, L_qq^-T) per group, 2 kGS^2 each; -1: none
  const double* H;      // [M][L0][n][n] (the discrete form's Hh)
  const double* betaf;  // [L0][L]
  const double* cdiag;  // [L+M]
  const double* scale;  // [L+M]
  const int* basis;     // [Nt][2] tiled basis (p, q)
  const int* hm_by_h;   // CSR of active (m,h) pair ids, per h: [L0 + 1] offsets ...
  const int* hm_ids;    // ... into this list of global pair ids
  const int* hm_m;      // ... and the m of each of those pairs
  const int* pq2b;      // [n][n]: basis index of entry (p, q) (symmetric)
  const int* h_by_m;    // CSR per derivative block m: [M + 1] offsets ...
  const int* h_list;    // ... into this list of h with H_{h,m} != 0
};

struct BlkDesc {
  int sys, j, n, pad;
  int64_t off;      // arena offset of the block (same for every block array)
};

// one active (m, h) pair: H_{h,m} != 0
struct HMPair {
  int sys, m, h, n;
  int64_t offY;     // scratch for H W (B operator)
  int64_t offA2;    // pre-product A2 = X H^T (A1 = Z^-1 H^T lives in a side table)
};

// one active (m, h, h2) with h <= h2 for the Schur pre-products
struct HM2 {
  int sys, m, h, h2, n, pad;
  int64_t offA3, offA4;   // H_h X H_h2^T and H_h Z^-1 H_h2^T
  int64_t srcA1, srcA2;   // A1[m][h2], A2[m][h2]
};

// one term of the Schur expansion for a pair (h, h2): the Kronecker factor
// T[b,c] U[d,a] summed over the symmetric components.
struct KTerm {
  int64_t offT, offU;   // arena offsets
  double coef;          // multiplies T
  int tT, tU;           // 1 = read transposed
};

struct AsmTile {
  int sys, h, h2, rg, cg, kbeg, kcnt, pad;
};

// host-side list of group pairs of the tiled basis for one n
struct BasisInfo {
  int n, NG, ngp;
  std::vector<int> pairs;      // [Nt][2]
  std::vector<int> gp_g1, gp_g2, gp_off, gp_size;
};

BasisInfo make_basis(int n);

}  // namespace psdp

struct psdp_sdp {
  int n, l, da, dp, d1, d2;
  int form;   // PSDP_FORM_*
  int bo;     // order of every block of the SDP: n, or 2n for the discrete form
  int L0, L, M, Na, Nt, nb;
  int64_t K, Kpad;
  double delta, eps;
  int paper_literal;
  std::vector<int> Wp, WL, WM, Wa;   // exponent tables [count][l]
  std::vector<uint8_t> bmask;        // [L0][L] beta_{h,j} != 0
  std::vector<uint8_t> hmask;        // [M][L0] H_{h,m} != 0
  psdp::BasisInfo basis;
  std::vector<double> betaf;         // host copies of the device set-up
  std::vector<double> cdiag_h, scale_h;
  int device;
  std::shared_ptr<void> dmem;   // device block, shared by the handles of one set-up call
  size_t dbytes;                // this handle's part of it
  double* dA;
  int64_t* dbeta;
  int64_t* dcoef;
  double* dH;
  double* dHh;       // discrete form: [M][L0][2n][2n] [[-b/2 I, -H], [0, -b/2 I]]; else dH
  double* dbetaf;
  double* dscale;
  double* dcdiag;
  int* dbasis;
};

namespace psdp {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define PSDP_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return ::psdp::fail(PSDP_EDEVICE, std::string(#call) + ": " +           \
                                            hipGetErrorString(e_));          \
  } while (0)

int64_t round_up(int64_t x, int64_t m);

// Schur Cholesky / triangular solve launches (chol.hip)
void launch_chol_diag(hipStream_t st, const SysDesc* sys, int* flags, const double* Lam,
                      double* Ldiag, double* Linv, const int* ssys, int cnt, int p);
void launch_chol_trsm(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                      const double* Linv, const int* ssys, const int* spre, int cnt, int total,
                      int p);
void launch_chol_update_wide(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                             const int* ssys, const int* spre, int cnt, int total, int p, int mode);
void launch_chol_update(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag,
                        double* Linv, const int* ssys, const int* spre, int cnt, int total, int p);
void launch_chol_fused(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                       double* PB, const int* ssys, const int* spre, int cnt, int total, int p);
void launch_chol_left(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                      const int* ssys, const int* spre, int cnt, int total, int j);
void launch_cholinv_tile(hipStream_t st, int nblk, const BlkDesc* blks, int* flags, const double* Z,
                         double* Zi);
void launch_certificate_tile(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                             const int* flags, const double* Q, int iters, double* out);
void launch_ladder_tile(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags, const double* V,
                        const double* dV, double rho, double frac, int len, int* kout);
void launch_chol_look(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                      const int* hsys, const int* hpre, int hcnt, int htot, const int* lsys, const int* lpre,
                      int lcnt, int ltot, int p);
void launch_trsv_ginv(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* Linv,
                      double* Ginv, int m, int phase);
void launch_trsv_gfinish(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                         const int* spre, int cnt, int total, const double* Linv, double* Ginv);
void launch_trsv_gapply(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                        const int* spre, int cnt, int total, const double* Ginv, const double* vin,
                        double* vout, int q, int backward);
void launch_trsv_gfwd(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* z, double* r,
                      int q);
void launch_trsv_gbwd(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* x, double* z,
                      int q);
void launch_trsv_small(hipStream_t st, int nsmall, const SysDesc* sys, const int* flags,
                       const int* small_ids, const double* Lam, const double* Linv,
                       const double* rhs, double* x);
constexpr int kSmallN = 16;   // blocks up to this order take the packed small-block kernels
constexpr int kSmallP = 32;   // systems with at most this many Schur tiles solve in one launch
constexpr int kSG = 16;      // panels per group of the tiled triangular solves
constexpr int kGS = kSG * kNB;   // rows of such a group
static_assert((kSG & (kSG - 1)) == 0, "the group inverses double block sizes");

// engine entry used by the public solve / eval calls
int solve_batch(psdp_sdp* const* sdps, int count, const psdp_opts* opts, psdp_result* res,
                bool noalloc = false);
int eval_newton(psdp_sdp* sdp, const double* X, const double* Z, const double* y, double* Zi,
                double* BTy, double* BX, double* Lam, double* LamL, double* sol, int chol_panels,
                int chol_subpanels, hipStream_t stream);
int eval_ladder(psdp_sdp* sdp, const double* V, const double* dV, const psdp_opts* o,
                double* step, int* kstar);
int eval_schur(psdp_sdp* sdp, const double* X, const double* Z, int precision, double* Lam,
               hipStream_t st);

}  // namespace psdp
