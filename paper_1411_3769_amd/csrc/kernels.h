// Launch wrappers of the per-iteration kernels (kernels.hip).
#pragma once

#include "internal.h"

namespace psdp {

void launch_cholinv(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                    int* flags, const double* Z, double* Zi);
void launch_ladder(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                   const int* flags, const double* V, const double* dV, double rho, double frac,
                   int len, int* kout);
void launch_ladder2(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                    const int* flags, const double* X, const double* dX, const double* Z,
                    const double* dZ, double rho, double frac, int len, int* koutX, int* koutZ);
void launch_steps_update_y(hipStream_t st, const SysDesc* sys, int S, int maxK, int* flags, const int* koutX,
                           const int* koutZ, double rho, double* sc, double* y, const double* dyh,
                           const double* dyb);
void launch_ladder_step(hipStream_t st, const SysDesc* sys, int S, int* flags, const int* kout,
                        double rho, int slot, double* sc);
void launch_gemm_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                        const double* sc, const double* A, int tA, const double* B, int tB,
                        double* C, double alpha, int aslot, const double* D, double beta,
                        int bslot, int nmin, int tiles = 1);
void launch_make_G(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                   const double* Cf, const double* S, const double* Z, double* G, int nskip = 0);
void launch_axpby(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags, double a,
                  const double* A, double b, const double* B, double* out, int nskip = 0);
void launch_symmetrize(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                       const double* W, double* out, int nskip = 0);
void launch_combine(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                    const double* dXh, const double* dXb, double* dX, const double* dZh,
                    const double* dZb, double* dZ, int nskip = 0);
void launch_update_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                          const double* sc, double* X, const double* dX, double* Z,
                          const double* dZ);
void launch_block_red(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                      const double* Cf, const double* X, const double* Z, const double* G,
                      double* red);
void launch_sys_finalize(hipStream_t st, int S, const SysDesc* sys, const int* flags,
                         const double* red, const double* y, const double* BX, double sigma,
                         double* sc);
void launch_form_P(hipStream_t st, int total, const SysDesc* sys, const int* flags,
                   const int* own_pre, int S, const double* y, double* Pm, int nskip);
void launch_BT_pblk(hipStream_t st, int n, const BlkDesc* pblks, const SysDesc* sys,
                    const int* flags, const double* Pm, double* out, int nskip);
void launch_BT_small(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys, const int* flags,
                     const double* y, double* out, const double* Cf = nullptr, const double* Z = nullptr,
                     double* G = nullptr);
void launch_BT_dblk(hipStream_t st, int n, const BlkDesc* dblks, const SysDesc* sys,
                    const int* flags, const double* Pm, double* out, int nmin, int tiles = 1);
void launch_B_Y(hipStream_t st, int np, const HMPair* pairs, const SysDesc* sys,
                const int* flags, const double* W, double* arena, const BlkDesc* blks, int nmin,
                int tiles = 1);
void launch_B_reduce(hipStream_t st, int totalK, const SysDesc* sys, const int* flags,
                     const int* own_pre, int S, const HMPair* pairs, const double* W,
                     const double* arena, const BlkDesc* blks, double* out, double asub, int nskip);
void launch_B_small(hipStream_t st, int totL0, const SysDesc* sys, const int* flags, const int* own_pre,
                    int S, const double* W, double* out, double asub);
void launch_pre12(hipStream_t st, int np, const HMPair* pairs, const SysDesc* sys,
                  const int* flags, const double* Zi, const double* X, double* arena,
                  const BlkDesc* blks, const int64_t* offA1, int nmin, int tiles = 1);
void launch_pre34(hipStream_t st, int nq, const HM2* q, const SysDesc* sys, const int* flags,
                  double* arena, int nmin, int tiles = 1);
void launch_assemble_pair(hipStream_t st, int ntiles, int maxn, const AsmTile* tiles,
                          const KTerm* terms, const SysDesc* sys, const int* flags,
                          const double* arena, double* Lam, int prec, double* rscr);
void launch_assemble_grp(hipStream_t st, int ntiles, const AsmTile* tiles, const KTerm* terms,
                         const SysDesc* sys, const int* flags, const int* gpinfo,
                         const double* arena, double* Lam, const int64_t* gpoff, int prec);
bool use_small(int nmax);

void launch_sym_ZAX_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                          const double* Zi, const double* A, const double* X, double* W1);
void launch_pred_dir_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                           const double* sc, const double* S1, const double* Gm, const double* Zi,
                           const double* X, double* dZh, double* dXh, double* Wc, double* W1);
void launch_corr_dir_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                           const double* Zi, const double* dZb, const double* X, const double* Wc,
                           const double* dXh, const double* dZh, double* dX, double* dZ);
void launch_pre12_small(hipStream_t st, int np, int nmax, const HMPair* pairs, const SysDesc* sys,
                        const int* flags, const double* Zi, const double* X, double* arena,
                        const BlkDesc* blks, const int64_t* offA1);
void launch_pre34_small(hipStream_t st, int nq, int nmax, const HM2* q, const SysDesc* sys,
                        const int* flags, double* arena);
void launch_init_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys, double* X,
                        double* Z, double* Cf);
void launch_warm_init(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                      const int* flags, const double* W, const double* cert, const double* logx,
                      double theta, double* X, double* Z);
void launch_warm_center(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                        const double* Zi, const double* logx, double* X);
void launch_block_logtrace(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                           const double* X, double* out);
void launch_park(hipStream_t st, int S, int* flags, int mode);
void launch_ir_check(hipStream_t st, int S, const SysDesc* sys, int* flags, const double* r,
                     const double* rhs, double* sc, int k, int kmax, int first_solve);
void launch_vec_axpby(hipStream_t st, int S, const SysDesc* sys, const int* flags, double a,
                      double* x, double b, const double* y);
void launch_pad_identity(hipStream_t st, int S, const SysDesc* sys, double* Lam);
void launch_mehrotra(hipStream_t st, int S, int nblk, const SysDesc* sys, const BlkDesc* blks,
                     const int* flags, const int* koutX, const int* koutZ, double rho, double sigma0,
                     const double* X, const double* dXs, const double* Z, const double* dZh,
                     const double* Zi, double* red, double* sc, double* Wc, double* W1);
void launch_schur_shift(hipStream_t st, int S, const SysDesc* sys, const int* flags, const double* shf,
                        double* Lam, double* sc);
void launch_certificate(hipStream_t st, int nblk, int maxn, const BlkDesc* blks,
                        const SysDesc* sys, const int* flags, const double* Q, int iters,
                        double* out);

void launch_lift(hipStream_t st, int S, const SysDesc* sys, const int* flags, const double* yin,
                 double* yout);
void launch_sub_tD(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                   const int* flags, const double* yp, double* out);
void launch_B_phase1(hipStream_t st, int S, const SysDesc* sys, const int* flags,
                     const BlkDesc* blks, const double* W, double* out, double asub);
void launch_gemm_scaled(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                        const int* flags, const double* A, const double* B, double* C, int tiles = 1);
void launch_lam_phase1(hipStream_t st, int S, int maxK, const SysDesc* sys, const int* flags,
                       const BlkDesc* blks, const double* W, const double* v, double* Lam);
void launch_phase1_vectors(hipStream_t st, int S, const SysDesc* sys, const int* flags, double* yp,
                           double* eK);

}  // namespace psdp
