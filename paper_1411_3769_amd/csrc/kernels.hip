// Per-iteration kernels of the interior-point method (Section IV, Alg. 2)
// over a batch of systems: block factorisations, the operators B and B^T
// (eq. AT with eq. Aij), the Schur complement assembly (eq. T2) and the
// step-length ladder.  Every block kernel runs one workgroup per n x n block
// of every system still active; blocks of all systems share one arena
// layout, so X, Z, Z^{-1}, G, ... of block b all live at blk[b].off.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devcommon.h"
#include "internal.h"
#include "kernels.h"

namespace psdp {

#define ACTIVE_OR_RETURN(s) \
  if (!(flags[(s)] & F_ACTIVE)) return

// Z_j -> Z_j^{-1} = L^{-T} L^{-1} through the in-LDS Cholesky factor.
__global__ void __launch_bounds__(256) k_cholinv(const BlkDesc* __restrict__ blks, int* flags,
                                                 const double* __restrict__ Z, double* Zi, int nmax) {
  extern __shared__ double sm[];
  __shared__ int fl;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kSmallN || bd.n > nmax) return;   // k_cholinv16 / k_cholinv_tile
  ACTIVE_OR_RETURN(bd.sys);
  const int n = bd.n, nn = n * n;
  const double* Zb = Z + bd.off;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) sm[e] = Zb[e];
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  wg_potrf(sm, n, n, &fl);
  if (threadIdx.x == 0 && fl) atomicOr(&flags[bd.sys], F_ZFAIL);
  wg_trtri_lower(sm, n, n);
  double* out = Zi + bd.off;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (j < i) continue;
    double acc = 0.0;
    for (int k = j; k < n; ++k) acc += sm[k * n + i] * sm[k * n + j];
    out[i * n + j] = acc;
    out[j * n + i] = acc;
  }
}

// Z_j^{-1} for blocks of order <= 16, sixteen lanes per block (sixteen blocks
// per workgroup), all in registers: lane r holds row r of Z (identity past
// n).  Z = L L^T with every column scaled by the Newton reciprocal square
// root of its pivot; lane c then forms column c of X = L^{-1} by forward
// substitution, and Z^{-1} = X^T X row by row (terms in ascending k, so the
// result is exactly symmetric).  Row values travel by DPP row broadcasts.
__global__ void __launch_bounds__(256) k_cholinv16(const BlkDesc* __restrict__ blks, int nblk,
                                                   int* flags, const double* __restrict__ Z,
                                                   double* Zi) {
  const int b = blockIdx.x * 16 + (int)(threadIdx.x >> 4), r = threadIdx.x & 15;
  if (b >= nblk) return;
  const BlkDesc bd = blks[b];
  if (bd.n > kSmallN) return;   // k_cholinv
  if (!(flags[bd.sys] & F_ACTIVE)) return;
  const int n = bd.n;
  const double* Zb = Z + bd.off;
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = (r < n && c < n) ? Zb[r * n + c] : (r == c ? 1.0 : 0.0);
  // lower Cholesky factor, row r of L in a; rs[k] = 1 / L[k][k]
  double rs[16];
  bool bad = false;
  static_for<16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double d = row_bcast16<k>(a[k]);
    const bool bb = !(d > 0.0) || !isfinite(d);
    bad = bad || bb;
    d = bb ? 1.0 : d;
    rs[k] = rsqrt_nr(d);
    const double lrk = r >= k ? a[k] * rs[k] : 0.0;
    a[k] = lrk;
    static_for<16>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c > k) {
        const double lck = row_bcast16<c>(lrk);
        a[c] = r >= c ? a[c] - lrk * lck : a[c];
      }
    });
  });
  if (bad && r == 0) atomicOr(&flags[bd.sys], F_ZFAIL);
  // column r of X = L^{-1}: x[i] = (delta_{ir} - sum_{m<i} L[i][m] x[m]) / L[i][i]
  double x[16];
  static_for<16>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    double acc = r == i ? 1.0 : 0.0;
    static_for<i>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      acc -= row_bcast16<i>(a[m]) * x[m];
    });
    x[i] = acc * rs[i];
  });
  // row r of X^T X: sum over k >= c of X[k][r] X[k][c]
  double* out = Zi + bd.off;
  static_for<16>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    double acc = 0.0;
    static_for<16>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k >= c) acc += x[k] * row_bcast16<c>(x[k]);
    });
    if (r < n && c < n) out[r * n + c] = acc;
  });
}

// Step-length ladder (reading of the paper's "standard line-search" that
// keeps X and Z positive semidefinite): r_0 = 1, r_{k+1} = rho r_k; block b
// records the first k at which V_b + (r_k / frac) dV_b passes Cholesky, -1
// if none up to len.  The trial matrix is formed with a separate multiply
// and add.
__global__ void __launch_bounds__(256) k_ladder(const BlkDesc* __restrict__ blks,
                                                const int* __restrict__ flags,
                                                const double* __restrict__ V,
                                                const double* __restrict__ dV, double rho,
                                                double frac, int len, int* kout, int nmax) {
  extern __shared__ double sm[];
  __shared__ int fl;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kSmallN || bd.n > nmax) return;   // k_ladder16 / k_ladder_tile
  if (!(flags[bd.sys] & F_ACTIVE)) {
    if (threadIdx.x == 0) kout[blockIdx.x] = 0;
    return;
  }
  const int n = bd.n, nn = n * n;
  const double* Vb = V + bd.off;
  const double* dVb = dV + bd.off;
  double r = 1.0;
  int found = -1;
  for (int k = 0; k <= len; ++k) {
    const double t = r / frac;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) sm[e] = __dadd_rn(Vb[e], __dmul_rn(t, dVb[e]));
    if (threadIdx.x == 0) fl = 0;
    __syncthreads();
    wg_potrf(sm, n, n, &fl);
    const int f = fl;
    __syncthreads();
    if (!f) {
      found = k;
      break;
    }
    r = r * rho;
  }
  if (threadIdx.x == 0) kout[blockIdx.x] = found;
}

// The same ladder for blocks of order <= 16, sixteen lanes per block
// (sixteen blocks per workgroup): lane r holds row r of the block (identity
// past n) and the rungs are tried in order with the row Cholesky test (the
// first rung passes in most iterations).  With nset = 2 the grid covers a
// second, independent ladder (V2, dV2 -> kout2) over the same blocks.
__global__ void __launch_bounds__(256) k_ladder16(const BlkDesc* __restrict__ blks, int nblk,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ V1,
                                                  const double* __restrict__ dV1, double rho,
                                                  double frac, int len, int* kout1, int nset,
                                                  const double* __restrict__ V2,
                                                  const double* __restrict__ dV2, int* kout2) {
  const int vb = blockIdx.x * 16 + (int)(threadIdx.x >> 4), r = threadIdx.x & 15;
  if (vb >= nset * nblk) return;
  const bool second = vb >= nblk;
  const int b = second ? vb - nblk : vb;
  const double* V = second ? V2 : V1;
  const double* dV = second ? dV2 : dV1;
  int* kout = second ? kout2 : kout1;
  const BlkDesc bd = blks[b];
  if (bd.n > kSmallN) return;   // k_ladder
  if (!(flags[bd.sys] & F_ACTIVE)) {
    if (r == 0) kout[b] = 0;
    return;
  }
  const int n = bd.n;
  double v0[16], dv[16];
  bool in[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    in[c] = c <= r && r < n;
    v0[c] = in[c] ? V[bd.off + r * n + c] : (r == c ? 1.0 : 0.0);
    dv[c] = in[c] ? dV[bd.off + r * n + c] : 0.0;
  }
  int found = -1;
  double rk = 1.0;
  for (int k = 0; k <= len; ++k) {
    const double t = rk / frac;
    double tv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) tv[c] = in[c] ? __dadd_rn(v0[c], __dmul_rn(t, dv[c])) : v0[c];
    if (rows_chol_ok16(tv, r)) {
      found = k;
      break;
    }
    rk = rk * rho;
  }
  if (r == 0) kout[b] = found;
}

// Per system: k* = max over blocks of the first passing rung; the step is
// r_{k*} (repeated multiplication, as the oracle does).  One wave per system.
__global__ void __launch_bounds__(256) k_ladder_step(const SysDesc* __restrict__ sys, int S, int* flags,
                                                     const int* __restrict__ kout, double rho, int slot,
                                                     double* sc) {
  const int s = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= S) return;
  if (!(flags[s] & F_ACTIVE)) return;
  const int blk0 = sys[s].blk0, nb = sys[s].nb;
  int kmax = 0, bad = 0;
  for (int j = lane; j < nb; j += 64) {
    const int k = kout[blk0 + j];
    bad |= k < 0;
    kmax = k > kmax ? k : kmax;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int ko = __shfl_xor(kmax, m);
    kmax = ko > kmax ? ko : kmax;
    bad |= __shfl_xor(bad, m);
  }
  if (lane != 0) return;
  double r = 1.0;
  for (int k = 0; k < kmax; ++k) r = r * rho;
  if (bad) {
    flags[s] |= F_LADDERFAIL;
    r = 0.0;
  }
  sc[s * kNSC + slot] = r;
}

// Both step lengths and the y update (eq. y), one wave per system and
// kYChunk entries of its y (grid dimension y): for each ladder, the step is
// rho^{k*} with k* the largest first passing rung over the system's blocks
// (repeated multiplication), 0 with F_LADDERFAIL if a block found none; S_TP
// from koutX, S_TD from koutZ (written by the chunk-0 wave; every wave
// derives the same values); then, unless the Newton system or a ladder
// failed, y += t_D (dy^ + dy_bar) on the wave's chunk.
constexpr int kYChunk = 256;
__global__ void __launch_bounds__(256) k_steps_update_y(const SysDesc* __restrict__ sys, int S, int* flags,
                                                        const int* __restrict__ koutX,
                                                        const int* __restrict__ koutZ, double rho,
                                                        double* sc, double* y,
                                                        const double* __restrict__ dyh,
                                                        const double* __restrict__ dyb) {
  const int s = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= S) return;
  const int f0 = flags[s];
  if (!(f0 & F_ACTIVE)) return;
  const SysDesc& sd = sys[s];
  const int blk0 = sd.blk0, nb = sd.nb;
  int kx = 0, kz = 0, bx = 0, bz = 0;
  for (int j = lane; j < nb; j += 64) {
    const int a = koutX[blk0 + j], c = koutZ[blk0 + j];
    bx |= a < 0;
    bz |= c < 0;
    kx = a > kx ? a : kx;
    kz = c > kz ? c : kz;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int ox = __shfl_xor(kx, m), oz = __shfl_xor(kz, m);
    kx = ox > kx ? ox : kx;
    kz = oz > kz ? oz : kz;
    bx |= __shfl_xor(bx, m);
    bz |= __shfl_xor(bz, m);
  }
  double tp = 1.0, td = 1.0;
  for (int k = 0; k < kx; ++k) tp = tp * rho;
  for (int k = 0; k < kz; ++k) td = td * rho;
  if (bx) tp = 0.0;
  if (bz) td = 0.0;
  if (lane == 0 && blockIdx.y == 0) {
    if (bx || bz) flags[s] = f0 | F_LADDERFAIL;
    sc[s * kNSC + S_TP] = tp;
    sc[s * kNSC + S_TD] = td;
  }
  if ((f0 & F_LAMFAIL) || bx || bz) return;
  const int kend = min(sd.K, (int)(blockIdx.y + 1) * kYChunk);
  for (int k = (int)blockIdx.y * kYChunk + lane; k < kend; k += 64) {
    const int64_t o = sd.voff + k;
    const double d = dyh[o] + dyb[o];
    y[o] = y[o] + td * d;
  }
}

// C_b = a op(A_b) op(B_b) + c D_b with a = alpha * sc[aslot], c = beta * sc[bslot]
// (slots < 0 mean 1).
__global__ void __launch_bounds__(256) k_gemm_blocks(const BlkDesc* __restrict__ blks,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ sc,
                                                     const double* A, int tA, const double* B,
                                                     int tB, double* C, double alpha, int aslot,
                                                     const double* D, double beta, int bslot,
                                                     int nmin) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n < nmin) return;
  double a = alpha, c = beta;
  if (aslot >= 0) a *= sc[bd.sys * kNSC + aslot];
  if (bslot >= 0) c *= sc[bd.sys * kNSC + bslot];
  wg_gemm_part(bd.n, A + bd.off, tA, B + bd.off, tB, C + bd.off, a, D ? D + bd.off : nullptr, c, sA, sB,
               blockIdx.y, gridDim.y);
}

// G = C - S + Z (eq. G with S = B^T(y))
__global__ void k_make_G(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                         const double* __restrict__ Cf, const double* __restrict__ S,
                         const double* __restrict__ Z, double* G, int nskip) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n <= nskip) return;   // k_BT_small's epilogue
  const int nn = bd.n * bd.n;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t o = bd.off + e;
    G[o] = Cf[o] - S[o] + Z[o];
  }
}

// out = a * A + b * B (elementwise over blocks)
__global__ void k_axpby(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                        double a, const double* __restrict__ A, double b,
                        const double* __restrict__ B, double* out, int nskip) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n <= nskip) return;   // the fused small-block kernels
  const int nn = bd.n * bd.n;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t o = bd.off + e;
    out[o] = a * A[o] + b * B[o];
  }
}

// out = (W + W^T) / 2 (out may alias W: each thread owns the pair (i,j),(j,i))
__global__ void k_symmetrize(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                             const double* W, double* out, int nskip) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n <= nskip) return;   // the fused small-block kernels
  const int n = bd.n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (j < i) continue;
    const double v = 0.5 * (W[bd.off + i * n + j] + W[bd.off + j * n + i]);
    out[bd.off + i * n + j] = v;
    out[bd.off + j * n + i] = v;
  }
}

// dX = sym(dXh + dXb), dZ = dZh + dZb
__global__ void k_combine(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                          const double* __restrict__ dXh, const double* __restrict__ dXb,
                          double* dX, const double* __restrict__ dZh,
                          const double* __restrict__ dZb, double* dZ, int nskip) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n <= nskip) return;   // k_corr_dir_small
  const int n = bd.n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const int64_t o = bd.off + e, ot = bd.off + j * n + i;
    const double sij = dXh[o] + dXb[o];
    const double sji = dXh[ot] + dXb[ot];
    dX[o] = 0.5 * (sij + sji);
    dZ[o] = dZh[o] + dZb[o];
  }
}

// X += tp dX, Z += td dZ (skipped when the Newton system or ladder failed)
__global__ void k_update_blocks(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                                const double* __restrict__ sc, double* X,
                                const double* __restrict__ dX, double* Z,
                                const double* __restrict__ dZ) {
  const BlkDesc bd = blks[blockIdx.x];
  const int f = flags[bd.sys];
  if (!(f & F_ACTIVE) || (f & (F_LAMFAIL | F_LADDERFAIL))) return;
  const double tp = sc[bd.sys * kNSC + S_TP], td = sc[bd.sys * kNSC + S_TD];
  const int nn = bd.n * bd.n;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t o = bd.off + e;
    X[o] = X[o] + tp * dX[o];
    Z[o] = Z[o] + td * dZ[o];
  }
}

// y += td (dyh + dyb)
// per-block partial sums: <C,X>, <Z,X>, ||G||^2, ||C||^2
__global__ void __launch_bounds__(256) k_block_red(const BlkDesc* __restrict__ blks,
                                                   const int* __restrict__ flags,
                                                   const double* __restrict__ Cf,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ Z,
                                                   const double* __restrict__ G, double* red) {
  __shared__ double s4[4][256];
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const int nn = bd.n * bd.n;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t o = bd.off + e;
    a0 += Cf[o] * X[o];
    a1 += Z[o] * X[o];
    a2 += G[o] * G[o];
    a3 += Cf[o] * Cf[o];
  }
  s4[0][threadIdx.x] = a0;
  s4[1][threadIdx.x] = a1;
  s4[2][threadIdx.x] = a2;
  s4[3][threadIdx.x] = a3;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s4[q][threadIdx.x] += s4[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) red[blockIdx.x * 4 + threadIdx.x] = s4[threadIdx.x][0];
}

__device__ inline double wg_sum256(double v, double* sbuf) {
  sbuf[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sbuf[threadIdx.x] += sbuf[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sbuf[0];
  __syncthreads();
  return r;
}

// NaN-propagating maximum (a NaN anywhere gives NaN)
__device__ inline double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ inline double wg_max256(double v, double* sbuf) {
  sbuf[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sbuf[threadIdx.x] = nanmax(sbuf[threadIdx.x], sbuf[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = sbuf[0];
  __syncthreads();
  return r;
}

// Per system: objectives, residual norms, gaps and mu (fixed summation order).
__global__ void __launch_bounds__(256) k_sys_finalize(const SysDesc* __restrict__ sys,
                                                      const int* __restrict__ flags,
                                                      const double* __restrict__ red,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ BX,
                                                      double sigma, double* sc) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  double c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  for (int j = threadIdx.x; j < sd.nb; j += blockDim.x) {
    const double* r = red + (int64_t)(sd.blk0 + j) * 4;
    c0 += r[0];
    c1 += r[1];
    c2 += r[2];
    c3 += r[3];
  }
  const double phi = wg_sum256(c0, sb);
  const double trzx = wg_sum256(c1, sb);
  const double g2 = wg_sum256(c2, sb);
  const double cc2 = wg_sum256(c3, sb);
  double py = 0, pr = 0, pb = 0, pa = 0;
  for (int k = threadIdx.x; k < sd.K; k += blockDim.x) {
    const double yk = y[sd.voff + k], bk = BX[sd.voff + k];
    double ak;
    if (sd.mode == 0) ak = 1.0; else ak = (k == sd.K - 1) ? -1.0 : 0.0;
    py += ak * yk;
    pr += (bk - ak) * (bk - ak);
    pb += bk * bk;
    pa += ak * ak;
  }
  const double psi = wg_sum256(py, sb);
  const double rr = wg_sum256(pr, sb);
  const double bb = wg_sum256(pb, sb);
  const double aa = wg_sum256(pa, sb);
  if (threadIdx.x == 0) {
    double* o = sc + s * kNSC;
    o[S_PHI] = phi;
    o[S_PSI] = psi;
    o[S_TRZX] = trzx;
    o[S_PINF] = sqrt(rr) / (1.0 + sqrt(aa));
    o[S_DINF] = sqrt(g2) / (1.0 + sqrt(cc2));
    o[S_GAPABS] = fabs(psi - phi);
    const double den = fmax(fabs(psi), fabs(phi));
    o[S_GAPREL] = den > 0 ? fabs(psi - phi) / den : fabs(psi - phi);
    o[S_NORMBX] = sqrt(bb);
    o[S_MU] = sigma * trzx / (double)(sd.nb * sd.n);
  }
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------

// P_h = V_h(y): one workgroup per (system, h); grid = sum_s L0_s (owner table)
__global__ void k_form_P(const SysDesc* __restrict__ sys, const int* __restrict__ flags,
                         const int* __restrict__ own_pre, int S, const double* __restrict__ y,
                         double* Pm, int nskip) {
  const int s = find_owner(own_pre, S, blockIdx.x);
  const int h = blockIdx.x - own_pre[s];
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  if (sd.n <= nskip) return;   // k_BT_small
  const int n = sd.n, nbs = sd.nbas;
  double* P = Pm + sd.poff + (int64_t)h * n * n;
  const double* yh = y + sd.voff + (int64_t)h * sd.Nt;
  for (int b = threadIdx.x; b < sd.Nt; b += blockDim.x) {
    const int p = sd.basis[2 * b], q = sd.basis[2 * b + 1];
    const double v = yh[b];
    for (int c = 0; c < sd.copies; ++c) {   // discrete form: blockdiag(P_h, P_h)
      const int pc = p + c * nbs, qc = q + c * nbs;
      P[pc * n + qc] = v;
      P[qc * n + pc] = v;
    }
  }
  if (sd.copies > 1)   // the off-diagonal copies stay zero
    for (int e = threadIdx.x; e < nbs * nbs; e += blockDim.x) {
      const int r = e / nbs, c = e % nbs;
      P[r * n + nbs + c] = 0.0;
      P[(nbs + r) * n + c] = 0.0;
    }
}

// P-blocks of B^T(y): out_j = sum_h beta_{h,j} P_h (ascending h)
__global__ void k_BT_pblk(const BlkDesc* __restrict__ pblks, const SysDesc* __restrict__ sys,
                          const int* __restrict__ flags, const double* __restrict__ Pm,
                          double* out, int nskip) {
  const BlkDesc bd = pblks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n <= nskip) return;   // k_BT_small
  const SysDesc sd = sys[bd.sys];
  const int nn = bd.n * bd.n;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    double acc = 0.0;
    for (int h = 0; h < sd.L0; ++h) {
      const double b = sd.betaf[h * sd.L + bd.j];
      if (b != 0.0) acc += b * Pm[sd.poff + (int64_t)h * nn + e];
    }
    out[bd.off + e] = acc;
  }
}

// derivative blocks of B^T(y), first part: Q = sum_h P_h H_{h,m} over the h
// with H_{h,m} != 0 (gamma_m >= h), the block's 64 x 64 tiles shared out over
// the grid's y dimension; k_BT_dsym then forms out = -(Q + Q^T)
__global__ void __launch_bounds__(256) k_BT_dblk(const BlkDesc* __restrict__ dblks,
                                                 const SysDesc* __restrict__ sys,
                                                 const int* __restrict__ flags,
                                                 const double* __restrict__ Pm, double* out,
                                                 int nmin) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const BlkDesc bd = dblks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n < nmin) return;
  const SysDesc sd = sys[bd.sys];
  const int n = bd.n, nn = n * n;
  const int m = bd.j - sd.L;
  double* O = out + bd.off;
  const int c0 = sd.h_by_m[m], c1 = sd.h_by_m[m + 1];
  if (c0 == c1) {
    if (blockIdx.y == 0)
      for (int e = threadIdx.x; e < nn; e += blockDim.x) O[e] = 0.0;
    return;
  }
  for (int c = c0; c < c1; ++c) {
    const int h = sd.h_list[c];
    const double* Hm = sd.H + ((int64_t)m * sd.L0 + h) * nn;
    wg_gemm_part(n, Pm + sd.poff + (int64_t)h * nn, 0, Hm, 0, O, 1.0, c == c0 ? nullptr : O, 1.0, sA, sB,
                 blockIdx.y, gridDim.y);
  }
}

// derivative blocks of B^T(y), second part: out = -(Q + Q^T) in place
__global__ void __launch_bounds__(256) k_BT_dsym(const BlkDesc* __restrict__ dblks,
                                                 const int* __restrict__ flags, double* out, int nmin) {
  const BlkDesc bd = dblks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  if (bd.n < nmin) return;
  const int n = bd.n, nn = n * n;
  double* O = out + bd.off;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (j < i) continue;
    const double v = -(O[i * n + j] + O[j * n + i]);
    O[i * n + j] = v;
    O[j * n + i] = v;
  }
}

// B operator, first stage: Y = H_{h,m} W_{L+m} for every active (m, h) pair
__global__ void __launch_bounds__(256) k_B_Y(const HMPair* __restrict__ pairs,
                                             const SysDesc* __restrict__ sys,
                                             const int* __restrict__ flags,
                                             const double* __restrict__ W, double* arena,
                                             const BlkDesc* __restrict__ blks, int nmin) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const HMPair pr = pairs[blockIdx.x];
  ACTIVE_OR_RETURN(pr.sys);
  if (pr.n < nmin) return;
  const SysDesc sd = sys[pr.sys];
  const int n = pr.n, nn = n * n;
  const double* Hm = sd.H + ((int64_t)pr.m * sd.L0 + pr.h) * nn;
  const BlkDesc bd = blks[sd.blk0 + sd.L + pr.m];
  wg_gemm_part(n, Hm, 0, W + bd.off, 0, arena + pr.offY, 1.0, nullptr, 0.0, sA, sB, blockIdx.y, gridDim.y);
}

// B operator, second stage: four lanes per (system, k = (h, b)), each taking
// every fourth term of both sums, then added across the four:
// out_k = sum_{j<L} beta_{h,j} <E_b, W_j> - 2 sum_m <E_b, Y_{m,h}> - a_k * asub
// (W symmetric).  Grid over 4 sum_s K_s (owner table of prefixes).
__global__ void __launch_bounds__(256) k_B_reduce(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const int* __restrict__ own_pre, int S,
                                                  const HMPair* __restrict__ pairs,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ arena,
                                                  const BlkDesc* __restrict__ blks, double* out,
                                                  double asub, int nskip) {
  const int gq = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = gq >> 2, qd = gq & 3;
  const int s = find_owner(own_pre, S, g);
  const SysDesc* sd = sys + s;
  const int k = g - own_pre[s];
  // systems with blocks of order <= nskip are left to k_B_small
  const bool live = k < sd->K && (flags[s] & F_ACTIVE) && sd->n > nskip;
  double acc = 0.0, dsum = 0.0;
  if (live) {
    const int n = sd->n, Nt = sd->Nt, L = sd->L;
    const int h = k / Nt, b = k - h * Nt;
    const int p = sd->basis[2 * b], q = sd->basis[2 * b + 1];
    // tr(E_b S) over the basis matrix's diagonal copies (two in the
    // discrete form's blocks of order 2 nbas)
    const int e1 = p * n + q, e2 = q * n + p;
    const int sh = sd->copies > 1 ? sd->nbas * (n + 1) : 0;
    for (int j = qd; j < L; j += 4) {
      const double bt = sd->betaf[h * L + j];
      const double* Wj = W + blks[sd->blk0 + j].off;
      double w = p == q ? Wj[e1] : Wj[e1] + Wj[e2];
      if (sh) w += p == q ? Wj[e1 + sh] : Wj[e1 + sh] + Wj[e2 + sh];
      acc += bt != 0.0 ? bt * w : 0.0;
    }
    for (int c = sd->hm_by_h[h] + qd; c < sd->hm_by_h[h + 1]; c += 4) {
      const double* Y = arena + pairs[sd->hm_ids[c]].offY;
      dsum += (p == q ? Y[e1] : Y[e1] + Y[e2]);
      if (sh) dsum += (p == q ? Y[e1 + sh] : Y[e1 + sh] + Y[e2 + sh]);
    }
  }
  // every lane of the quad takes part in the shuffles
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  dsum += __shfl_xor(dsum, 1);
  dsum += __shfl_xor(dsum, 2);
  if (!live || qd != 0) return;
  acc -= 2.0 * dsum;
  out[sd->voff + k] = sd->mode == 0 ? acc - asub : acc;
}

// ---------------------------------------------------------------------------
// Schur complement (Alg. 2 eq. T2) through the rank expansion of each block:
// with E = e_a e_b^T, E' = e_c e_d^T and H = H_{h,m}, H' = H_{h2,m}
//   tr((H^T E + E H) Zi (H'^T E' + E' H') X) = sum_t T_t[b,c] U_t[d,a]
//   (T,U) in {(Zi H'^T, X H^T), (Zi, H' X H^T), (H Zi H'^T, X), (H Zi, H' X)},
// and P-blocks give beta_{h,j} beta_{h2,j} Zi[b,c] X[d,a].
// ---------------------------------------------------------------------------

// A1 = Z^{-1}_m H_h^T, A2 = X_m H_h^T
__global__ void __launch_bounds__(256) k_pre12(const HMPair* __restrict__ pairs,
                                               const SysDesc* __restrict__ sys,
                                               const int* __restrict__ flags,
                                               const double* __restrict__ Zi,
                                               const double* __restrict__ X, double* arena,
                                               const BlkDesc* __restrict__ blks,
                                               const int64_t* __restrict__ offA1, int nmin) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const HMPair pr = pairs[blockIdx.x];
  ACTIVE_OR_RETURN(pr.sys);
  if (pr.n < nmin) return;
  const SysDesc sd = sys[pr.sys];
  const int n = pr.n, nn = n * n;
  const double* Hm = sd.H + ((int64_t)pr.m * sd.L0 + pr.h) * nn;
  const BlkDesc bd = blks[sd.blk0 + sd.L + pr.m];
  wg_gemm_part(n, Zi + bd.off, 0, Hm, 1, arena + offA1[blockIdx.x], 1.0, nullptr, 0.0, sA, sB, blockIdx.y,
               gridDim.y);
  wg_gemm_part(n, X + bd.off, 0, Hm, 1, arena + pr.offA2, 1.0, nullptr, 0.0, sA, sB, blockIdx.y, gridDim.y);
}

// A3 = H_h A2[m][h2] = H_h X H_h2^T,  A4 = H_h A1[m][h2] = H_h Zi H_h2^T
__global__ void __launch_bounds__(256) k_pre34(const HM2* __restrict__ q,
                                               const SysDesc* __restrict__ sys,
                                               const int* __restrict__ flags, double* arena, int nmin) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const HM2 pr = q[blockIdx.x];
  ACTIVE_OR_RETURN(pr.sys);
  if (pr.n < nmin) return;
  const SysDesc sd = sys[pr.sys];
  const int n = pr.n, nn = n * n;
  const double* Hh = sd.H + ((int64_t)pr.m * sd.L0 + pr.h) * nn;
  wg_gemm_part(n, Hh, 0, arena + pr.srcA2, 0, arena + pr.offA3, 1.0, nullptr, 0.0, sA, sB, blockIdx.y,
               gridDim.y);
  wg_gemm_part(n, Hh, 0, arena + pr.srcA1, 0, arena + pr.offA4, 1.0, nullptr, 0.0, sA, sB, blockIdx.y,
               gridDim.y);
}

// ---------------------------------------------------------------------------
// certificate: Q_j = B^T(y)_j; pass = Cholesky succeeds; margin_j =
// lambda_min(Q_j) / s_j by bisection on the Cholesky of Q_j - tau s_j I.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_certificate(const BlkDesc* __restrict__ blks,
                                                     const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ Q, int iters,
                                                     double* out, int nmax) {
  extern __shared__ double sm[];
  __shared__ int fl;
  __shared__ double fro;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kSmallN || bd.n > nmax) return;   // k_certificate16 / k_certificate_tile
  ACTIVE_OR_RETURN(bd.sys);
  const SysDesc sd = sys[bd.sys];
  const int n = bd.n, nn = n * n;
  const double sj = sd.scale[bd.j];
  const double* Qb = Q + bd.off;
  if (threadIdx.x == 0) {
    double f = 0;
    for (int e = 0; e < nn; ++e) f += Qb[e] * Qb[e];
    fro = sqrt(f);
  }
  double lo = 0, hi = 0;
  int pass0 = 0;
  for (int it = -1; it < iters; ++it) {
    double tau;
    if (it < 0) tau = 0.0;
    else tau = 0.5 * (lo + hi);
    __syncthreads();
    const double shift = tau * sj;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
      const int i = e / n, j = e % n;
      sm[e] = (i == j) ? Qb[e] - shift : Qb[e];
    }
    if (threadIdx.x == 0) fl = 0;
    __syncthreads();
    wg_potrf(sm, n, n, &fl);
    const int ok = !fl;
    __syncthreads();
    if (it < 0) {
      pass0 = ok;
      const double bnd = fro / sj + 1.0;
      if (ok) { lo = 0.0; hi = bnd; } else { lo = -bnd; hi = 0.0; }
    } else {
      if (ok) lo = tau; else hi = tau;
    }
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x * 2 + 0] = pass0;
    out[blockIdx.x * 2 + 1] = 0.5 * (lo + hi);
  }
}

// The same certificate for blocks of order <= 16, sixteen lanes per block
// (lane r holds row r): the block stays in registers (identity past n, never
// shifted) and each bisection step is one row Cholesky test.
__global__ void __launch_bounds__(256) k_certificate16(const BlkDesc* __restrict__ blks, int nblk,
                                                       const SysDesc* __restrict__ sys,
                                                       const int* __restrict__ flags,
                                                       const double* __restrict__ Q, int iters,
                                                       double* out) {
  const int b = blockIdx.x * 16 + (int)(threadIdx.x >> 4), r = threadIdx.x & 15;
  if (b >= nblk) return;
  const BlkDesc bd = blks[b];
  if (bd.n > kSmallN) return;   // k_certificate
  if (!(flags[bd.sys] & F_ACTIVE)) return;
  const int n = bd.n;
  const double sj = sys[bd.sys].scale[bd.j];
  double q[16], fg[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const bool in = r < n && c < n;
    q[c] = in ? Q[bd.off + r * n + c] : (r == c ? 1.0 : 0.0);
    if (in) fg[c >> 2] += q[c] * q[c];
  }
  // ||Q||_F: column quarters paired (0, 2), (1, 3), then rows by xor 8, 4, 2, 1
  double f = (fg[0] + fg[2]) + (fg[1] + fg[3]);
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) f += __shfl_xor(f, m);
  const double fro = sqrt(f);
  double lo = 0, hi = 0;
  int pass0 = 0;
  for (int it = -1; it < iters; ++it) {
    const double tau = it < 0 ? 0.0 : 0.5 * (lo + hi);
    const double shift = tau * sj;
    double tv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) tv[c] = (r == c && r < n) ? q[c] - shift : q[c];
    const bool ok = rows_chol_ok16(tv, r);
    if (it < 0) {
      pass0 = ok;
      const double bnd = fro / sj + 1.0;
      if (ok) { lo = 0.0; hi = bnd; } else { lo = -bnd; hi = 0.0; }
    } else {
      if (ok) lo = tau; else hi = tau;
    }
  }
  if (r == 0) {
    out[b * 2 + 0] = pass0;
    out[b * 2 + 1] = 0.5 * (lo + hi);
  }
}

// Schur matrices: rows/columns past K carry the identity.
__global__ void k_pad_identity(const SysDesc* __restrict__ sys, double* Lam) {
  const SysDesc sd = sys[blockIdx.x];
  for (int i = sd.K + threadIdx.x; i < sd.Kpad; i += blockDim.x)
    Lam[sd.loff + (int64_t)i * sd.Kpad + i] = 1.0;
}


// ---------------------------------------------------------------------------
// Mehrotra's centring parameter (option): from the ladders of the predictor
// directions, t_p^a and t_d^a (first passing rungs as for the step lengths),
// mu_aff = tr((Z + t_d^a dZ^)(X + t_p^a sym dX^)) / m and
// sigma = min(1, max(0, (mu_aff / mu)^3)) with mu = tr(ZX) / m; the fixed
// sigma stays if either ladder finds no step.  The corrector right-hand side
// formed with the fixed sigma is moved to the new mu: W += (mu' - mu) Z^-1.
// ---------------------------------------------------------------------------

// one wave per system: predictor step lengths into S_TPA / S_TDA (-1: none)
__global__ void __launch_bounds__(256) k_mehrotra_steps(const SysDesc* __restrict__ sys, int S,
                                                        const int* __restrict__ flags,
                                                        const int* __restrict__ koutX,
                                                        const int* __restrict__ koutZ, double rho,
                                                        double* sc) {
  const int s = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= S) return;
  if (!(flags[s] & F_ACTIVE)) return;
  const int blk0 = sys[s].blk0, nb = sys[s].nb;
  int kx = 0, kz = 0, bad = 0;
  for (int j = lane; j < nb; j += 64) {
    const int a = koutX[blk0 + j], c = koutZ[blk0 + j];
    bad |= (a < 0) | (c < 0);
    kx = a > kx ? a : kx;
    kz = c > kz ? c : kz;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int ox = __shfl_xor(kx, m), oz = __shfl_xor(kz, m);
    kx = ox > kx ? ox : kx;
    kz = oz > kz ? oz : kz;
    bad |= __shfl_xor(bad, m);
  }
  if (lane != 0) return;
  double tp = 1.0, td = 1.0;
  for (int k = 0; k < kx; ++k) tp = tp * rho;
  for (int k = 0; k < kz; ++k) td = td * rho;
  sc[(size_t)s * kNSC + S_TPA] = bad ? -1.0 : tp;
  sc[(size_t)s * kNSC + S_TDA] = bad ? -1.0 : td;
}

// per block: red[4 blk] = tr((Z + td dZ^)(X + tp dXs)), both factors symmetric
__global__ void __launch_bounds__(256) k_mehrotra_trace(const BlkDesc* __restrict__ blks,
                                                        const int* __restrict__ flags,
                                                        const double* __restrict__ sc,
                                                        const double* __restrict__ X,
                                                        const double* __restrict__ dXs,
                                                        const double* __restrict__ Z,
                                                        const double* __restrict__ dZh, double* red) {
  __shared__ double sb[256];
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const double tp = sc[(size_t)bd.sys * kNSC + S_TPA], td = sc[(size_t)bd.sys * kNSC + S_TDA];
  double a = 0.0;
  for (int e = threadIdx.x; e < bd.n * bd.n; e += blockDim.x) {
    const int64_t o = bd.off + e;
    a += (Z[o] + td * dZh[o]) * (X[o] + tp * dXs[o]);
  }
  a = wg_sum256(a, sb);
  if (threadIdx.x == 0) red[(int64_t)blockIdx.x * 4] = a;
}

// per system: sigma, the new mu and its change
__global__ void __launch_bounds__(256) k_mehrotra_sigma(const SysDesc* __restrict__ sys,
                                                        const int* __restrict__ flags,
                                                        const double* __restrict__ red,
                                                        double sigma0, double* sc) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  double a = 0.0;
  for (int j = threadIdx.x; j < sd.nb; j += blockDim.x) a += red[(int64_t)(sd.blk0 + j) * 4];
  a = wg_sum256(a, sb);
  if (threadIdx.x == 0) {
    double* o = sc + (size_t)s * kNSC;
    const double m = (double)(sd.nb * sd.n);
    const double trzx = o[S_TRZX];
    double sigma = sigma0;
    if (o[S_TPA] >= 0.0 && o[S_TDA] >= 0.0) {
      const double q = (a / m) / (trzx / m);
      sigma = fmin(1.0, fmax(0.0, q * q * q));
    }
    const double mu = sigma * trzx / m;
    o[S_MUDELTA] = mu - o[S_MU];
    o[S_MU] = mu;
  }
}

// Wc += delta Z^-1 and W1 += delta Z^-1 (W1 = sym Wc; Z^-1 is symmetric)
__global__ void __launch_bounds__(256) k_mu_fix(const BlkDesc* __restrict__ blks,
                                                const int* __restrict__ flags,
                                                const double* __restrict__ sc,
                                                const double* __restrict__ Zi, double* Wc, double* W1) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const double dm = sc[(size_t)bd.sys * kNSC + S_MUDELTA];
  for (int e = threadIdx.x; e < bd.n * bd.n; e += blockDim.x) {
    const int64_t o = bd.off + e;
    Wc[o] = Wc[o] + dm * Zi[o];
    W1[o] = W1[o] + dm * Zi[o];
  }
}

void launch_mehrotra(hipStream_t st, int S, int nblk, const SysDesc* sys, const BlkDesc* blks,
                     const int* flags, const int* koutX, const int* koutZ, double rho, double sigma0,
                     const double* X, const double* dXs, const double* Z, const double* dZh,
                     const double* Zi, double* red, double* sc, double* Wc, double* W1) {
  if (S <= 0 || nblk <= 0) return;
  k_mehrotra_steps<<<(S + 3) / 4, 256, 0, st>>>(sys, S, flags, koutX, koutZ, rho, sc);
  k_mehrotra_trace<<<nblk, 256, 0, st>>>(blks, flags, sc, X, dXs, Z, dZh, red);
  k_mehrotra_sigma<<<S, 256, 0, st>>>(sys, flags, red, sigma0, sc);
  k_mu_fix<<<nblk, 256, 0, st>>>(blks, flags, sc, Zi, Wc, W1);
}

// Diagonal shift of the Schur matrix before it is factored, for the systems
// flagged F_SHIFTED (the retry after a failed FP64 factorisation, Alg. 2 root
// step 1): tau = shf[s] max_i Lambda_ii over the system's K unknowns (the
// assembled matrix, phase-I transform included), Lambda_ii += tau.  One
// workgroup per system; sc receives max diag and tau.
__global__ void __launch_bounds__(256) k_schur_shift(const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ shf, double* Lam,
                                                     double* sc) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  const int f = flags[s];
  if (!(f & F_ACTIVE) || !(f & F_SHIFTED)) return;
  const SysDesc sd = sys[s];
  double* A = Lam + sd.loff;
  const int64_t ld1 = sd.Kpad + 1;
  double m = -INFINITY;
  for (int i = threadIdx.x; i < sd.K; i += blockDim.x) m = nanmax(m, A[i * ld1]);
  m = wg_max256(m, sb);
  const double tau = shf[s] * m;
  for (int i = threadIdx.x; i < sd.K; i += blockDim.x) A[i * ld1] = A[i * ld1] + tau;
  if (threadIdx.x == 0) {
    sc[(size_t)s * kNSC + S_DIAGMAX] = m;
    sc[(size_t)s * kNSC + S_TAU] = tau;
  }
}

void launch_schur_shift(hipStream_t st, int S, const SysDesc* sys, const int* flags, const double* shf,
                        double* Lam, double* sc) {
  if (S > 0) k_schur_shift<<<S, 256, 0, st>>>(sys, flags, shf, Lam, sc);
}

// ---------------------------------------------------------------------------
// phase-I margin SDP (max t s.t. B^T(y) - t D >= 0, a^T y = 1, with y_K
// eliminated): operators and Schur complement expressed through the paper's.
// ---------------------------------------------------------------------------

// yout = (u, -sum u) for phase-I systems (u = the first K-1 entries of yin),
// a plain copy for the others.
__global__ void __launch_bounds__(256) k_lift(const SysDesc* __restrict__ sys,
                                              const int* __restrict__ flags,
                                              const double* __restrict__ yin, double* yout) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  const double* a = yin + sd.voff;
  double* b = yout + sd.voff;
  if (sd.mode == 0) {
    for (int k = threadIdx.x; k < sd.K; k += blockDim.x) b[k] = a[k];
    return;
  }
  double part = 0.0;
  for (int k = threadIdx.x; k < sd.K - 1; k += blockDim.x) {
    b[k] = a[k];
    part += a[k];
  }
  const double tot = wg_sum256(part, sb);
  if (threadIdx.x == 0) b[sd.K - 1] = -tot;
}

// out_j -= t s_j I for phase-I systems (t = the last entry of y')
__global__ void k_sub_tD(const BlkDesc* __restrict__ blks, const SysDesc* __restrict__ sys,
                         const int* __restrict__ flags, const double* __restrict__ yp,
                         double* out) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const SysDesc sd = sys[bd.sys];
  if (sd.mode != 1) return;
  const double t = yp[sd.voff + sd.K - 1];
  const double sj = sd.scale[bd.j];
  for (int i = threadIdx.x; i < bd.n; i += blockDim.x) out[bd.off + i * bd.n + i] -= t * sj;
}

// B'(W) from B(W) in place: out_i -= out_{K-1} (i < K-1),
// out_{K-1} = -sum_j s_j tr(W_j); then the phase-I a' = (0,..,0,-1) enters
// as out_{K-1} += asub.
__global__ void __launch_bounds__(256) k_B_phase1(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const BlkDesc* __restrict__ blks,
                                                  const double* __restrict__ W, double* out,
                                                  double asub) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  if (sd.mode != 1) return;
  double* o = out + sd.voff;
  const double last = o[sd.K - 1];
  double part = 0.0;
  for (int e = threadIdx.x; e < sd.nb * sd.n; e += blockDim.x) {
    const int j = e / sd.n, i = e % sd.n;
    const BlkDesc bd = blks[sd.blk0 + j];
    part += sd.scale[j] * W[bd.off + i * sd.n + i];
  }
  const double tr = wg_sum256(part, sb);   // all threads have read `last`
  for (int k = threadIdx.x; k < sd.K - 1; k += blockDim.x) o[k] -= last;
  if (threadIdx.x == 0) o[sd.K - 1] = -tr + asub;
}

// W_j = s_j Z^{-1}_j X_j
__global__ void __launch_bounds__(256) k_gemm_scaled(const BlkDesc* __restrict__ blks,
                                                     const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const double* A, const double* B, double* C) {
  __shared__ double sA[16 * 64];
  __shared__ double sB[16 * 64];
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const SysDesc sd = sys[bd.sys];
  if (sd.mode != 1) return;
  wg_gemm_part(bd.n, A + bd.off, 0, B + bd.off, 0, C + bd.off, sd.scale[bd.j], nullptr, 0.0, sA, sB,
               blockIdx.y, gridDim.y);
}

// Lambda'_ij = Lambda_ij - Lambda_{K-1,i} - Lambda_{K-1,j} + Lambda_{K-1,K-1}
// for i, j < K-1 (lower triangle read, both triangles written); one workgroup
// per row i (grid.x over rows, grid.y over systems).
__global__ void k_lam_phase1_a(const SysDesc* __restrict__ sys, const int* __restrict__ flags,
                               double* Lam) {
  const int s = blockIdx.y, i = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  if (sd.mode != 1 || i >= sd.K - 1) return;
  double* A = Lam + sd.loff;
  const int64_t ld = sd.Kpad;
  const int64_t last = (int64_t)(sd.K - 1) * ld;
  const double cK = A[last + sd.K - 1];
  const double ci = A[last + i];
  for (int j = threadIdx.x; j <= i; j += blockDim.x) {
    const double v = A[(int64_t)i * ld + j] - ci - A[last + j] + cK;
    A[(int64_t)i * ld + j] = v;
    if (j != i) A[(int64_t)j * ld + i] = v;
  }
}

// last row/column: Lambda'_{t,j} = -(v_j - v_{K-1}), Lambda'_{t,t} =
// sum_j s_j tr(W_j) with W_j = s_j Z^{-1}_j X_j and v = B(W).
__global__ void __launch_bounds__(256) k_lam_phase1_b(const SysDesc* __restrict__ sys,
                                                      const int* __restrict__ flags,
                                                      const BlkDesc* __restrict__ blks,
                                                      const double* __restrict__ W,
                                                      const double* __restrict__ v, double* Lam) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  if (sd.mode != 1) return;
  double part = 0.0;
  for (int e = threadIdx.x; e < sd.nb * sd.n; e += blockDim.x) {
    const int j = e / sd.n, i = e % sd.n;
    part += sd.scale[j] * W[blks[sd.blk0 + j].off + i * sd.n + i];
  }
  const double tt = wg_sum256(part, sb);
  double* A = Lam + sd.loff;
  const int64_t ld = sd.Kpad;
  const double* vs = v + sd.voff;
  const double vK = vs[sd.K - 1];
  for (int j = threadIdx.x; j < sd.K - 1; j += blockDim.x) {
    const double val = -(vs[j] - vK);
    A[(int64_t)(sd.K - 1) * ld + j] = val;
    A[(int64_t)j * ld + sd.K - 1] = val;
  }
  if (threadIdx.x == 0) A[(int64_t)(sd.K - 1) * ld + sd.K - 1] = tt;
}

// phase-I starting point y' = (1/K, ..., 1/K, 0), and e_K for building C'.
__global__ void k_phase1_vectors(const SysDesc* __restrict__ sys, const int* __restrict__ flags,
                                 double* yp, double* eK) {
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  for (int k = threadIdx.x; k < sd.Kpad; k += blockDim.x) {
    yp[sd.voff + k] = k < sd.K - 1 ? 1.0 / sd.K : 0.0;
    eK[sd.voff + k] = k == sd.K - 1 ? 1.0 : 0.0;
  }
}


// ---------------------------------------------------------------------------
// Schur complement assembly on FP64 MFMA (v_mfma_f64_16x16x4: A 16x4,
// B 4x16; lane l supplies A[l%16][l/16] and B[l/16][l%16], and result
// register i of lane l holds D[4i + l/16][l%16], i = 0..3).
//
// For a pair (h, h2) the expansion terms k = (block, t) give
//   R[(b,c),(d,a)] = sum_k T_k[b,c] U_k[d,a]          (a product of the
// stacked, flattened T and U: rows n^2, columns n^2, inner dimension #k), and
//   Lambda[(p,q),(r,s)] = sum_{(a,b) in S(p,q)} sum_{(c,d) in S(r,s)} R[(b,c),(d,a)]
// with S(p,q) = {(p,q),(q,p)} (p != q) or {(p,p)}.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Reduced-precision forms (PR = 1: FP32, PR = 2: BF16) stage T and U
// rounded to the narrow type and accumulate in FP32; the gather and the
// Schur matrix stay FP64.  v_mfma_f32_16x16x4f32 takes A[l%16][l/16] and
// B[l/16][l%16]; v_mfma_f32_16x16x16bf16_1k takes A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16], j = 0..3; both return D[4(l/16)+i][l%16] in register i.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// double -> bf16 bits, through FP32, round to nearest even
__device__ inline unsigned short to_bf16(double x) {
  const float f = (float)x;
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <int PR> struct AsmPrec;
template <> struct AsmPrec<0> {
  typedef double stage_t; typedef v4d acc_t; static constexpr int KC = 4;
  static __device__ stage_t cvt(double x) { return x; }
};
template <> struct AsmPrec<1> {
  typedef float stage_t; typedef v4f acc_t; static constexpr int KC = 4;
  static __device__ stage_t cvt(double x) { return (float)x; }
};
template <> struct AsmPrec<2> {
  typedef unsigned short stage_t; typedef v4f acc_t; static constexpr int KC = 16;
  static __device__ stage_t cvt(double x) { return to_bf16(x); }
};

// One MFMA step; sA / sB point at the lane's first operand element, and
// successive k (bf16 only) are kstride apart.
template <int PR>
__device__ inline typename AsmPrec<PR>::acc_t asm_mfma(const typename AsmPrec<PR>::stage_t* sA,
                                                       const typename AsmPrec<PR>::stage_t* sB,
                                                       int kstride,
                                                       typename AsmPrec<PR>::acc_t c) {
  if constexpr (PR == 0) return mfma16(*sA, *sB, c);
  else if constexpr (PR == 1) return __builtin_amdgcn_mfma_f32_16x16x4f32(*sA, *sB, c, 0, 0, 0);
  else {
    v4s a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = (short)sA[j * kstride];
      b[j] = (short)sB[j * kstride];
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
}

// output row of result register i (16 x 16 tile)
template <int PR>
__device__ inline int asm_row(int lane, int i) {
  return PR == 0 ? 4 * i + (lane >> 4) : 4 * (lane >> 4) + i;
}

// Small n (n^2 <= 128): one workgroup of 8 waves per (system, h, h2) pair,
// the grid striding over pairs.  R = sum_k T_k (x) U_k (n^2 x n^2) is
// accumulated in registers (16 x 16 MFMA tiles dealt round-robin to the
// waves), then written out for the gather into Lambda.  Terms are staged
// kPairKS at a time: every thread owns one entry index (and its transpose)
// of T and U for a quarter of the stage's terms, fetches the next stage into
// registers while the current one is multiplied, and writes it to LDS after
// the barrier.  RL: R lives in LDS (overlaying the staging area), else in
// this workgroup's slot of global scratch.  TPW: MFMA tiles per wave, at
// least ceil(NT^2 / 8) for the batch's largest n; a wave's tiles past the
// system's last are computed on a duplicate and dropped, so the tile loop is
// branch-free.
constexpr int kPairKS = 16;
constexpr int kPairWaves = 8;

template <int PR, bool RL, int TPW>
__device__ __forceinline__ void assemble_pair(const AsmTile* __restrict__ tiles, int npt,
                                              const KTerm* __restrict__ terms,
                                              const SysDesc* __restrict__ sys,
                                              const int* __restrict__ flags,
                                              const double* __restrict__ arena, double* Lam,
                                              double* rscr, int rslot) {
  extern __shared__ double smem[];
  typedef AsmPrec<PR> AP;
  typedef typename AP::stage_t real;
  typedef typename AP::acc_t acc_t;
  constexpr int KC = AP::KC;
  constexpr int KS = kPairKS;
  constexpr int NQ = kPairWaves / 2;      // thread quarters of 128
  constexpr int KH = KS / NQ;             // terms per thread and stage
  constexpr int NTH = 64 * kPairWaves;
  double* R = RL ? smem : rscr + (int64_t)blockIdx.x * rslot;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qtr = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int idx = tid & 127;
  const int kq = lane >> 4, r16 = lane & 15;
  const int kb = PR == 2 ? 4 * kq : kq;
  for (int tix = blockIdx.x; tix < npt; tix += gridDim.x) {
    const AsmTile tl = tiles[tix];
    if (!(flags[tl.sys] & F_ACTIVE)) continue;
    if (((flags[tl.sys] & F_ASM32) != 0) != (PR != 0)) continue;
    const SysDesc sd = sys[tl.sys];
    // entry indices run over the basis order n, addresses over the block
    // order bo (the discrete form's terms are n x n blocks of 2n x 2n ones)
    const int n = sd.nbas, bo = sd.n, n2 = n * n;
    const int NT = (n2 + 15) / 16, n2p = NT * 16, ntiles = NT * NT;
    const int kcnt = tl.kcnt;
    const bool inb = idx < n2;
    const int ii = inb ? idx : 0;
    const int ib = ii / n, ic = ii - ib * n;
    const int iad = ib * bo + ic, itr = ic * bo + ib;
    real* sT = reinterpret_cast<real*>(smem);
    real* sU = sT + KS * n2p;
    // raw entries and the term's coefficient (0 past the last term); the
    // descriptors are read first and the entry loads are unconditional
    // (clamped), so that a whole stage is in flight at once
    double vT[KH], vU[KH], cf[KH];
    auto fetch = [&](int k0) {
      KTerm kt[KH];
#pragma unroll
      for (int j = 0; j < KH; ++j) kt[j] = terms[tl.kbeg + min(k0 + qtr + NQ * j, kcnt - 1)];
#pragma unroll
      for (int j = 0; j < KH; ++j) {
        vT[j] = arena[kt[j].offT + (kt[j].tT ? itr : iad)];
        vU[j] = arena[kt[j].offU + (kt[j].tU ? itr : iad)];
        cf[j] = k0 + qtr + NQ * j < kcnt ? kt[j].coef : 0.0;
      }
    };
    acc_t acc[TPW];
    int toff[TPW], uoff[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      acc[t] = acc_t{0, 0, 0, 0};
      const int id = min(wave + kPairWaves * t, ntiles - 1);
      const int ti = id / NT;
      toff[t] = ti * 16;
      uoff[t] = (id - ti * NT) * 16;
    }
    if (kcnt > 0) fetch(0);
    for (int k0 = 0; k0 < kcnt; k0 += KS) {
      __syncthreads();   // the previous stage (or pair) is no longer read
      if (idx < n2p) {
#pragma unroll
        for (int j = 0; j < KH; ++j) {
          const bool ok = inb && cf[j] != 0.0;
          sT[(qtr + NQ * j) * n2p + idx] = AP::cvt(ok ? cf[j] * vT[j] : 0.0);
          sU[(qtr + NQ * j) * n2p + idx] = AP::cvt(ok ? vU[j] : 0.0);
        }
      }
      __syncthreads();
      if (k0 + KS < kcnt) fetch(k0 + KS);
      // a partial last stage multiplies only the k-steps that hold terms
      const int kend = min(KS, kcnt - k0);
#pragma unroll 1
      for (int ks = 0; ks < kend; ks += KC) {
        const real* bT = sT + (ks + kb) * n2p + r16;
        const real* bU = sU + (ks + kb) * n2p + r16;
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = asm_mfma<PR>(bT + toff[t], bU + uoff[t], n2p, acc[t]);
      }
    }
    if (RL) __syncthreads();   // staging area becomes R
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      if (wave + kPairWaves * t < ntiles) {
        const int col = uoff[t] + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = toff[t] + asm_row<PR>(lane, i);
          if (row < n2 && col < n2) R[row * n2 + col] = (double)acc[t][i];
        }
      }
    }
    __syncthreads();
    const int Nt = sd.Nt;
    const int64_t ld = sd.Kpad;
    double* Lr = Lam + sd.loff;
    // Lambda[(h, b1), (h2, b2)] goes to its lower-triangle place
    // (h2 Nt + b2, h Nt + b1), the only triangle the factorisation reads;
    // consecutive threads take consecutive b1, i.e. consecutive columns
#pragma unroll 2
    for (int e = tid; e < Nt * Nt; e += NTH) {
      const int b2 = e / Nt, b1 = e - b2 * Nt;
      const int p = sd.basis[2 * b1], q = sd.basis[2 * b1 + 1];
      const int r = sd.basis[2 * b2], s = sd.basis[2 * b2 + 1];
      double v = R[(q * n + r) * n2 + s * n + p];
      if (r != s) v += R[(q * n + s) * n2 + r * n + p];
      if (p != q) {
        v += R[(p * n + r) * n2 + s * n + q];
        if (r != s) v += R[(p * n + s) * n2 + r * n + q];
      }
      const int64_t row = (int64_t)tl.h * Nt + b1, col = (int64_t)tl.h2 * Nt + b2;
      Lr[col * ld + row] = v;
    }
    if (!RL) __syncthreads();   // R is rewritten by the next pair
  }
}

// FP64 / FP32 operands: two workgroups per CU (4 waves a SIMD: at most 128
// registers a lane)
template <int PR, bool RL, int TPW>
__global__ void __launch_bounds__(512, 4) k_assemble_pair(const AsmTile* __restrict__ tiles, int npt,
                                                          const KTerm* __restrict__ terms,
                                                          const SysDesc* __restrict__ sys,
                                                          const int* __restrict__ flags,
                                                          const double* __restrict__ arena,
                                                          double* Lam, double* rscr, int rslot) {
  assemble_pair<PR, RL, TPW>(tiles, npt, terms, sys, flags, arena, Lam, rscr, rslot);
}

// BF16 operands (more registers for the k-groups of a stage) and n = 11
// (TPW 8): one workgroup per CU
template <int PR, bool RL, int TPW>
__global__ void __launch_bounds__(512) k_assemble_pair_1wg(const AsmTile* __restrict__ tiles, int npt,
                                                           const KTerm* __restrict__ terms,
                                                           const SysDesc* __restrict__ sys,
                                                           const int* __restrict__ flags,
                                                           const double* __restrict__ arena,
                                                           double* Lam, double* rscr, int rslot) {
  assemble_pair<PR, RL, TPW>(tiles, npt, terms, sys, flags, arena, Lam, rscr, rslot);
}

// General n: one workgroup per Schur tile (row group (g1,g2) of h, column
// group (g3,g4) of h2; groups of 8 indices).  A quarter of the waves (the
// c-th) accumulates one of the four symmetric components over the stacked
// terms,
//   Q1 = sum T[q,r] U[s,p],  Q2 = sum T[q,s] U[r,p],
//   Q3 = sum T[p,r] U[s,q],  Q4 = sum T[p,s] U[r,q],
// as a 64 x 64 MFMA product (rows (x,y), columns (z,u) of 8 x 8 indices), each
// wave 64 / (kGrpW / 4) of its columns; the four are added into an LDS tile in
// (p,q) x (r,s) order (Q3/Q4 only for p != q, Q2/Q4 only for r != s).
constexpr int kGrpW = 16;   // waves of a k_assemble_grp workgroup (4 components x kGrpW / 4)

// two workgroups per CU: kGrpW / 2 waves per SIMD
template <int PR>
__global__ void __launch_bounds__(64 * kGrpW) __attribute__((amdgpu_waves_per_eu(kGrpW / 2))) k_assemble_grp(const AsmTile* __restrict__ tiles,
                                                      const KTerm* __restrict__ terms,
                                                      const SysDesc* __restrict__ sys,
                                                      const int* __restrict__ flags,
                                                      const int* __restrict__ gpinfo_all,
                                                      const double* __restrict__ arena,
                                                      double* Lam,
                                                      const int64_t* __restrict__ gpoff) {
  typedef AsmPrec<PR> AP;
  typedef typename AP::stage_t real;
  typedef typename AP::acc_t acc_t;
  constexpr int KC = AP::KC;                 // depth of one MFMA
  constexpr int KS = PR == 2 ? 16 : 8;       // terms per LDS stage
  constexpr int WPC = kGrpW / 4;             // waves per component
  constexpr int NCT = 4 / WPC;               // 16-column tiles per wave
  constexpr int KH = KS / WPC;               // terms a thread stages per stage
  // two stage buffers (one multiplied while the next is written) and, after
  // the last product, the combined tile share one LDS block (two workgroups
  // fit a compute unit)
  constexpr int kOp = KS * 16 * 17;          // one operand of one stage
  constexpr int kStage = 4 * kOp * (int)sizeof(real), kTile = 64 * 65 * 8;
  __shared__ __align__(16) char smem[kStage > kTile ? kStage : kTile];
  real* const sbuf = reinterpret_cast<real*>(smem);   // T of buffer b at 2 b kOp, U after it
  double* sL = reinterpret_cast<double*>(smem);
  const AsmTile tl = tiles[blockIdx.x];
  ACTIVE_OR_RETURN(tl.sys);
  if (((flags[tl.sys] & F_ASM32) != 0) != (PR != 0)) return;
  if (tl.kcnt <= 0) return;   // (a pair without terms gets no tiles)
  const SysDesc sd = sys[tl.sys];
  const int n = sd.n, nbs = sd.nbas;   // block order (entry addresses), basis order (indices)
  const int* gp = gpinfo_all + gpoff[tl.sys];
  const int g1 = gp[tl.rg * 4 + 0], g2 = gp[tl.rg * 4 + 1], roff = gp[tl.rg * 4 + 2];
  const int g3 = gp[tl.cg * 4 + 0], g4 = gp[tl.cg * 4 + 1], coff = gp[tl.cg * 4 + 2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cpt = w / WPC, hh = w % WPC;   // component, column part
  // index offsets of the component's row pair (x, y) and column pair (z, u)
  const int xoff = cpt < 2 ? 8 : 0, yoff = (cpt & 1) ? 8 : 0;
  const int zoff = (cpt & 1) ? 0 : 8, uoff = cpt < 2 ? 0 : 8;
  // every thread stages entry (a, c) of T and of U for half of a stage's
  // terms (the half of its four waves)
  const int th = tid & 255, half = __builtin_amdgcn_readfirstlane(tid >> 8);   // staging part
  const int sa = th >> 4, sc = th & 15;
  const int ia = sa < 8 ? kTB * g1 + sa : kTB * g2 + (sa - 8);
  const int jc = sc < 8 ? kTB * g3 + sc : kTB * g4 + (sc - 8);
  const bool inb = ia < nbs && jc < nbs;
  const int iN = inb ? ia * n + jc : 0, iT = inb ? jc * n + ia : 0;
  // Stage st is multiplied from LDS buffer st % 2 while the registers holding
  // stage st + 1 are written to the other buffer and stage st + 2 is
  // fetched into them: the stage's term descriptors first, then every entry
  // load (clamped, unconditional, so that all are in flight together); the
  // coefficient (0 past the last term) is applied when the stage is written.
  // One barrier per stage: a buffer is rewritten only after every wave has
  // passed the barrier that ends its last product.
  double vT[KH], vU[KH], cf[KH];
  auto fetch = [&](int k0) {
    KTerm kt[KH];
    const int kf = k0 + half * KH;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) kt[kk] = terms[tl.kbeg + min(kf + kk, tl.kcnt - 1)];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      vT[kk] = arena[kt[kk].offT + (kt[kk].tT ? iT : iN)];
      vU[kk] = arena[kt[kk].offU + (kt[kk].tU ? iN : iT)];
      cf[kk] = kf + kk < tl.kcnt ? kt[kk].coef : 0.0;
    }
  };
  auto put = [&](int b) {
    real* dT = sbuf + 2 * b * kOp + half * KH * 272;
    real* dU = dT + kOp;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const bool ok = inb && cf[kk] != 0.0;
      dT[kk * 272 + sa * 17 + sc] = AP::cvt(ok ? cf[kk] * vT[kk] : 0.0);   // T[I_a][J_c]
      dU[kk * 272 + sc * 17 + sa] = AP::cvt(ok ? vU[kk] : 0.0);            // U[J_c][I_a]
    }
  };
  acc_t acc[4 * NCT];
#pragma unroll
  for (int t = 0; t < 4 * NCT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  const int kq = lane >> 4, r16 = lane & 15;
  fetch(0);
  put(0);
  fetch(KS);
  __syncthreads();
  for (int st = 0, k0 = 0; k0 < tl.kcnt; ++st, k0 += KS) {
    const int b = st & 1;
    put(b ^ 1);          // stage st + 1 (zeros past the end)
    fetch(k0 + 2 * KS);
    const real* sT = sbuf + 2 * b * kOp;
    const real* sU = sT + kOp;
    // a partial last stage multiplies only the k-steps that hold terms
    const int kend = min(KS, tl.kcnt - k0);
#pragma unroll
    for (int ks = 0; ks < KS; ks += KC) {
      if (ks >= kend) break;
      const int kb = ks + (PR == 2 ? 4 * kq : kq);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int xi = 2 * t + (r16 >> 3), yi = r16 & 7;
        const real* pa = sT + kb * 272 + (xoff + xi) * 17 + yoff + yi;
#pragma unroll
        for (int v = 0; v < NCT; ++v) {
          const int u = NCT * hh + v;
          const int zi = 2 * u + (r16 >> 3), ui = r16 & 7;
          const real* pb = sU + kb * 272 + (zoff + zi) * 17 + uoff + ui;
          acc[t * NCT + v] = asm_mfma<PR>(pa, pb, 272, acc[t * NCT + v]);
        }
      }
    }
    __syncthreads();
  }
  // combine the four components in LDS (the two waves of a component write
  // disjoint columns)
  const bool pqdiag = (g1 == g2), rsdiag = (g3 == g4);
  for (int ph = 0; ph < 4; ++ph) {
    __syncthreads();
    if (cpt == ph) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < NCT; ++v)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * t + asm_row<PR>(lane, i);
            const int col = 16 * (NCT * hh + v) + (lane & 15);
            const int xi = row >> 3, yi = row & 7, zi = col >> 3, ui = col & 7;
            int pi, qi, ri, si;
            if (cpt == 0) { pi = ui; qi = xi; ri = yi; si = zi; }
            else if (cpt == 1) { pi = ui; qi = xi; ri = zi; si = yi; }
            else if (cpt == 2) { pi = xi; qi = ui; ri = yi; si = zi; }
            else { pi = xi; qi = ui; ri = zi; si = yi; }
            const bool pq_same = pqdiag && pi == qi, rs_same = rsdiag && ri == si;
            double val = (double)acc[t * NCT + v][i];
            if ((cpt >= 2 && pq_same) || ((cpt & 1) && rs_same)) val = 0.0;
            double* dst = sL + (pi * 8 + qi) * 65 + ri * 8 + si;
            if (cpt == 0) *dst = val; else *dst += val;
          }
    }
  }
  __syncthreads();
  const int n1 = min(kTB, nbs - kTB * g1), n2s = min(kTB, nbs - kTB * g2);
  const int n3 = min(kTB, nbs - kTB * g3), n4 = min(kTB, nbs - kTB * g4);
  const int64_t ld = sd.Kpad;
  double* Lr = Lam + sd.loff;
  // every entry goes to its lower-triangle place (col, row) (a diagonal
  // tile covers its own transpose); consecutive threads take consecutive rows
  for (int e = tid; e < 4096; e += 64 * kGrpW) {
    const int coll = e >> 6, rowl = e & 63;
    const int pi = rowl >> 3, qi = rowl & 7, ri = coll >> 3, si = coll & 7;
    if (pi >= n1 || qi >= n2s || ri >= n3 || si >= n4) continue;
    if (pqdiag && qi < pi) continue;
    if (rsdiag && si < ri) continue;
    const int bi = pqdiag ? pi * n1 - pi * (pi - 1) / 2 + (qi - pi) : pi * n2s + qi;
    const int bj = rsdiag ? ri * n3 - ri * (ri - 1) / 2 + (si - ri) : ri * n4 + si;
    const int64_t row = (int64_t)tl.h * sd.Nt + roff + bi;
    const int64_t col = (int64_t)tl.h2 * sd.Nt + coff + bj;
    Lr[col * ld + row] = sL[rowl * 65 + coll];
  }
}


// ---------------------------------------------------------------------------
// Small blocks (n <= 16): G = 256 / nmax^2 products per workgroup, one output
// entry per thread.  Every thread first stages one entry of each operand in
// LDS (so each operand element is read from memory once, not n times), then
// forms its dot products from LDS.  Items whose order exceeds nmax belong to
// the general kernels and are skipped (each block takes the same kernel
// whatever the batch holds).
// ---------------------------------------------------------------------------
__device__ inline double dot_n(int n, int i, int j, const double* A, int tA, const double* B, int tB) {
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double a = tA ? A[k * n + i] : A[i * n + k];
    const double b = tB ? B[j * n + k] : B[k * n + j];
    acc += a * b;
  }
  return acc;
}

// this thread's item (li within the workgroup) and entry e
struct SmallSlot {
  int li, item, e, per;
  bool ok;
};

__device__ inline SmallSlot small_slot(int nmax, int G, int count) {
  SmallSlot t;
  t.per = nmax * nmax;
  t.li = (int)threadIdx.x / t.per;
  t.item = blockIdx.x * G + t.li;
  t.e = (int)threadIdx.x - t.li * t.per;
  t.ok = (int)threadIdx.x < G * t.per && t.item < count;
  return t;
}

// Fused chains of block products for blocks of order <= 16 (G blocks per
// workgroup, one thread per entry, operands and intermediates in LDS).  Each
// performs, entry for entry, the arithmetic of the launches it replaces.

// W1 = sym(Z^-1 A X): T = Z^-1 A, W = T X, W1 = (W + W^T) / 2
__global__ void __launch_bounds__(256) k_sym_ZAX_small(int nblk, int nmax, int G,
                                                       const BlkDesc* __restrict__ blks,
                                                       const int* __restrict__ flags,
                                                       const double* __restrict__ Zi,
                                                       const double* __restrict__ A,
                                                       const double* __restrict__ X, double* W1) {
  __shared__ double sZ[256], sA[256], sX[256], sT[256];
  SmallSlot t = small_slot(nmax, G, nblk);
  BlkDesc bd{};
  if (t.ok) {
    bd = blks[t.item];
    t.ok = (flags[bd.sys] & F_ACTIVE) && bd.n <= nmax && t.e < bd.n * bd.n;
  }
  const int base = t.li * t.per, n = bd.n;
  const int i = t.ok ? t.e / n : 0, j = t.ok ? t.e - i * n : 0;
  const int64_t o = bd.off + t.e;
  double *pz = sZ + base, *pa = sA + base, *px = sX + base, *pt = sT + base;
  if (t.ok) {
    pz[t.e] = Zi[o];
    pa[t.e] = A[o];
    px[t.e] = X[o];
  }
  __syncthreads();
  if (t.ok) pt[t.e] = 1.0 * dot_n(n, i, j, pz, 0, pa, 0);
  __syncthreads();
  if (t.ok) pa[t.e] = 1.0 * dot_n(n, i, j, pt, 0, px, 0);
  __syncthreads();
  if (t.ok) W1[o] = 0.5 * (pa[i * n + j] + pa[j * n + i]);
}

// predictor directions and the corrector's right-hand side:
// dZh = S1 - G, T = Z^-1 dZh, dXh = -T X - X, Wc = -T dXh + mu Z^-1,
// W1 = sym(Wc)
__global__ void __launch_bounds__(256) k_pred_dir_small(
    int nblk, int nmax, int G, const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
    const double* __restrict__ sc, const double* __restrict__ S1, const double* __restrict__ Gm,
    const double* __restrict__ Zi, const double* __restrict__ X, double* dZh, double* dXh,
    double* Wc, double* W1) {
  __shared__ double sZ[256], sX[256], sD[256], sT[256], sH[256], sC[256];
  SmallSlot t = small_slot(nmax, G, nblk);
  BlkDesc bd{};
  if (t.ok) {
    bd = blks[t.item];
    t.ok = (flags[bd.sys] & F_ACTIVE) && bd.n <= nmax && t.e < bd.n * bd.n;
  }
  const int base = t.li * t.per, n = bd.n;
  const int i = t.ok ? t.e / n : 0, j = t.ok ? t.e - i * n : 0;
  const int64_t o = bd.off + t.e;
  double *pz = sZ + base, *px = sX + base, *pd = sD + base, *pt = sT + base, *ph = sH + base,
         *pc = sC + base;
  if (t.ok) {
    pz[t.e] = Zi[o];
    px[t.e] = X[o];
    const double dz = -1.0 * Gm[o] + 1.0 * S1[o];
    pd[t.e] = dz;
    dZh[o] = dz;
  }
  __syncthreads();
  if (t.ok) pt[t.e] = 1.0 * dot_n(n, i, j, pz, 0, pd, 0);
  __syncthreads();
  if (t.ok) {
    double v = -1.0 * dot_n(n, i, j, pt, 0, px, 0);
    v += -1.0 * px[t.e];
    ph[t.e] = v;
    dXh[o] = v;
  }
  __syncthreads();
  if (t.ok) {
    const double mu = 1.0 * sc[bd.sys * kNSC + S_MU];
    double v = -1.0 * dot_n(n, i, j, pt, 0, ph, 0);
    v += mu * pz[t.e];
    pc[t.e] = v;
    Wc[o] = v;
  }
  __syncthreads();
  if (t.ok) W1[o] = 0.5 * (pc[i * n + j] + pc[j * n + i]);
}

// corrector directions and their sum with the predictor's:
// T = Z^-1 dZb, dXb = -T X + Wc, dX = sym(dXh + dXb), dZ = dZh + dZb
__global__ void __launch_bounds__(256) k_corr_dir_small(
    int nblk, int nmax, int G, const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
    const double* __restrict__ Zi, const double* __restrict__ dZb, const double* __restrict__ X,
    const double* __restrict__ Wc, const double* __restrict__ dXh, const double* __restrict__ dZh,
    double* dX, double* dZ) {
  __shared__ double sZ[256], sB[256], sX[256], sT[256], sS[256];
  SmallSlot t = small_slot(nmax, G, nblk);
  BlkDesc bd{};
  if (t.ok) {
    bd = blks[t.item];
    t.ok = (flags[bd.sys] & F_ACTIVE) && bd.n <= nmax && t.e < bd.n * bd.n;
  }
  const int base = t.li * t.per, n = bd.n;
  const int i = t.ok ? t.e / n : 0, j = t.ok ? t.e - i * n : 0;
  const int64_t o = bd.off + t.e;
  double *pz = sZ + base, *pb = sB + base, *px = sX + base, *pt = sT + base, *ps = sS + base;
  double zb = 0.0;
  if (t.ok) {
    pz[t.e] = Zi[o];
    zb = dZb[o];
    pb[t.e] = zb;
    px[t.e] = X[o];
  }
  __syncthreads();
  if (t.ok) pt[t.e] = 1.0 * dot_n(n, i, j, pz, 0, pb, 0);
  __syncthreads();
  if (t.ok) {
    double v = -1.0 * dot_n(n, i, j, pt, 0, px, 0);
    v += 1.0 * Wc[o];
    ps[t.e] = dXh[o] + v;
  }
  __syncthreads();
  if (t.ok) {
    dX[o] = 0.5 * (ps[i * n + j] + ps[j * n + i]);
    dZ[o] = dZh[o] + zb;
  }
}

// B(W) for systems whose blocks have order <= 16, one workgroup of four
// waves per (system, h), without per-pair products in the arena:
// S = sum_{j<L} beta_{h,j} W_j and R = sum over the (m, h) pairs of
// H_{h,m} W_{L+m} (a contraction over (m, k) on FP64 MFMA, operands read
// straight into the A/B lane layout, zero past n; each wave takes every
// fourth pair and every fourth j and keeps T_w = S_w - 2 R_w in the D
// layout), then for every basis pair b = (p, q) of h: out_{(h,b)} =
// T[p][q] + T[q][p] (T[p][p] if p = q) with T = sum_w T_w, less asub on the
// paper's SDP.
constexpr int kBG = 4;   // pairs whose operands one wave loads together

__global__ void __launch_bounds__(256) k_B_small(const SysDesc* __restrict__ sys,
                                                 const int* __restrict__ flags,
                                                 const int* __restrict__ own_pre, int S,
                                                 const double* __restrict__ W, double* out,
                                                 double asub) {
  __shared__ double sT[4][256];
  const int s = find_owner(own_pre, S, blockIdx.x);
  const int h = blockIdx.x - own_pre[s];
  ACTIVE_OR_RETURN(s);
  const SysDesc& sd = sys[s];
  const int n = sd.n;
  if (n > kSmallN) return;   // k_B_Y + k_B_reduce
  const int nn = n * n, L = sd.L, L0 = sd.L0;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const double* Ws = W + sd.boff;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  // R: pairs c0 + wv, c0 + wv + 4, ..., kBG of them per round
  const int c0 = sd.hm_by_h[h], c1 = sd.hm_by_h[h + 1];
  for (int cb = c0 + wv; cb < c1; cb += 4 * kBG) {
    double av[kBG][4], bv[kBG][4];
#pragma unroll
    for (int g = 0; g < kBG; ++g) {
      const int c = cb + 4 * g;
      const int m = sd.hm_m[min(c, c1 - 1)];
      const double* Hc = sd.H + ((int64_t)m * L0 + h) * nn;
      const double* Wc = Ws + (int64_t)(L + m) * nn;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int k = 4 * ks + kq;
        const bool ok = c < c1 && k < n && r16 < n;
        av[g][ks] = ok ? Hc[r16 * n + k] : 0.0;   // A[i][k], i = r16
        bv[g][ks] = ok ? Wc[k * n + r16] : 0.0;   // B[k][j], j = r16
      }
    }
#pragma unroll
    for (int g = 0; g < kBG; ++g)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        if (4 * ks < n) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g][ks], bv[g][ks], acc, 0, 0, 0);
  }
  // S at the D layout: rows 4q + kq, column r16; j' = wv, wv + 4, ...
  double sv[4] = {0.0, 0.0, 0.0, 0.0};
  {
    const double* bh = sd.betaf + (int64_t)h * L;
    for (int jb = wv; jb < L; jb += 16) {
      double w[4][4], bt[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = jb + 4 * u;
        bt[u] = jj < L ? bh[jj] : 0.0;
        const double* Wj = Ws + (int64_t)min(jj, L - 1) * nn;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 4 * q + kq;
          w[u][q] = row < n && r16 < n ? Wj[row * n + r16] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) sv[q] += bt[u] != 0.0 ? bt[u] * w[u][q] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sT[wv][(4 * q + kq) * 16 + r16] = sv[q] - 2.0 * acc[q];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < sd.Nt) {
    const int p = sd.basis[2 * t], q = sd.basis[2 * t + 1];
    auto T = [&](int a, int b) { return sT[0][a * 16 + b] + sT[1][a * 16 + b] + sT[2][a * 16 + b] + sT[3][a * 16 + b]; };
    double v = 0.0;
    for (int c = 0, o = 0; c < sd.copies; ++c, o += sd.nbas)   // diagonal copies of E_b
      v += p == q ? T(p + o, p + o) : T(p + o, q + o) + T(q + o, p + o);
    out[sd.voff + (int64_t)h * sd.Nt + t] = sd.mode == 0 ? v - asub : v;
  }
}

// B^T(y) for systems whose blocks have order <= 16, one wave per block
// (four per workgroup), reading P_h = V_h(y) straight from y through the
// (p, q) -> basis index table: P-blocks out_j = sum_h beta_{h,j} P_h
// (ascending h); derivative blocks Q = sum_{h : H_{h,m} != 0} P_h H_{h,m} on
// FP64 MFMA (ascending h), out = -(Q + Q^T) through the wave's LDS tile.
// With G given, also G = C - out + Z (eq. G) from the same registers.
__global__ void __launch_bounds__(256) k_BT_small(int nblk, const BlkDesc* __restrict__ blks,
                                                  const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ y, double* out,
                                                  const double* __restrict__ Cf,
                                                  const double* __restrict__ Zb, double* G) {
  __shared__ double sQ[4][256];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int b = blockIdx.x * 4 + wv;
  if (b >= nblk) return;
  const BlkDesc bd = blks[b];
  if (bd.n > kSmallN) return;   // k_form_P + k_BT_pblk + k_BT_dblk
  if (!(flags[bd.sys] & F_ACTIVE)) return;
  const SysDesc& sd = sys[bd.sys];
  const int n = bd.n, nn = n * n, L = sd.L, L0 = sd.L0, Nt = sd.Nt;
  const double* yv = y + sd.voff;
  double* O = out + bd.off;
  if (bd.j < L) {
    // entries e = lane + 64 u
    int ix[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) ix[u] = sd.pq2b[min(lane + 64 * u, nn - 1)];
    for (int h = 0; h < L0; ++h) {
      const double bt = sd.betaf[(int64_t)h * L + bd.j];
      if (bt == 0.0) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += ix[u] >= 0 ? bt * yv[(int64_t)h * Nt + ix[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane + 64 * u < nn) {
        const int64_t o = bd.off + lane + 64 * u;
        O[lane + 64 * u] = acc[u];
        if (G) G[o] = Cf[o] - acc[u] + Zb[o];
      }
    return;
  }
  const int m = bd.j - L;
  const int c0 = sd.h_by_m[m], c1 = sd.h_by_m[m + 1];
  // A[i][k] = P_h[i][k] = y[h Nt + pq2b[i n + k]], B[k][j] = H_{h,m}[k][j]
  int ia[4];
  bool oka[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + kq;
    ia[ks] = r16 < n && k < n ? sd.pq2b[r16 * n + k] : -1;
    oka[ks] = ia[ks] >= 0;   // (entries off the discrete form's diagonal copies are -1)
  }
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  for (int c = c0; c < c1; ++c) {
    const int h = sd.h_list[c];
    const double* Hm = sd.H + ((int64_t)m * L0 + h) * nn;
    double av[4], bv[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k = 4 * ks + kq;
      av[ks] = oka[ks] ? yv[(int64_t)h * Nt + ia[ks]] : 0.0;
      bv[ks] = k < n && r16 < n ? Hm[k * n + r16] : 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      if (4 * ks < n) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks], acc, 0, 0, 0);
  }
  double* q = sQ[wv];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[(4 * i + kq) * 16 + r16] = acc[i];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * i + kq;
    if (row < n && r16 < n) {
      const double v = -(acc[i] + q[r16 * 16 + row]);
      O[row * n + r16] = v;
      if (G) {
        const int64_t o = bd.off + row * n + r16;
        G[o] = Cf[o] - v + Zb[o];
      }
    }
  }
}

// A1 = Z^-1_m H_{m,h}^T, A2 = X_m H_{m,h}^T
__global__ void __launch_bounds__(256) k_pre12_small(int np, int nmax, int G,
                                                     const HMPair* __restrict__ pairs,
                                                     const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ Zi,
                                                     const double* __restrict__ X, double* arena,
                                                     const BlkDesc* __restrict__ blks,
                                                     const int64_t* __restrict__ offA1) {
  __shared__ double sZ[256], sX[256], sH[256];
  SmallSlot t = small_slot(nmax, G, np);
  HMPair pr{};
  if (t.ok) {
    pr = pairs[t.item];
    t.ok = (flags[pr.sys] & F_ACTIVE) && pr.n <= nmax && t.e < pr.n * pr.n;
  }
  const int n = pr.n, nn = n * n;
  double* pz = sZ + t.li * t.per;
  double* px = sX + t.li * t.per;
  double* ph = sH + t.li * t.per;
  if (t.ok) {
    const SysDesc* sd = sys + pr.sys;
    const BlkDesc bd = blks[sd->blk0 + sd->L + pr.m];
    pz[t.e] = Zi[bd.off + t.e];
    px[t.e] = X[bd.off + t.e];
    ph[t.e] = sd->H[((int64_t)pr.m * sd->L0 + pr.h) * nn + t.e];
  }
  __syncthreads();
  if (!t.ok) return;
  const int i = t.e / n, j = t.e - i * n;
  arena[offA1[t.item] + t.e] = dot_n(n, i, j, pz, 0, ph, 1);
  arena[pr.offA2 + t.e] = dot_n(n, i, j, px, 0, ph, 1);
}

// A3 = H_{m,h} A2[m][h2], A4 = H_{m,h} A1[m][h2]
__global__ void __launch_bounds__(256) k_pre34_small(int nq, int nmax, int G,
                                                     const HM2* __restrict__ q,
                                                     const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     double* arena) {
  __shared__ double sH[256], s2[256], s1[256];
  SmallSlot t = small_slot(nmax, G, nq);
  HM2 pr{};
  if (t.ok) {
    pr = q[t.item];
    t.ok = (flags[pr.sys] & F_ACTIVE) && pr.n <= nmax && t.e < pr.n * pr.n;
  }
  const int n = pr.n, nn = n * n;
  double* ph = sH + t.li * t.per;
  double* p2 = s2 + t.li * t.per;
  double* p1 = s1 + t.li * t.per;
  if (t.ok) {
    const SysDesc* sd = sys + pr.sys;
    ph[t.e] = sd->H[((int64_t)pr.m * sd->L0 + pr.h) * nn + t.e];
    p2[t.e] = arena[pr.srcA2 + t.e];
    p1[t.e] = arena[pr.srcA1 + t.e];
  }
  __syncthreads();
  if (!t.ok) return;
  const int i = t.e / n, j = t.e - i * n;
  arena[pr.offA3 + t.e] = dot_n(n, i, j, ph, 0, p2, 0);
  arena[pr.offA4 + t.e] = dot_n(n, i, j, ph, 0, p1, 0);
}

// x = a * x + b * y over the first K entries of every active system
__global__ void k_vec_axpby(const SysDesc* __restrict__ sys, const int* __restrict__ flags,
                            double a, double* x, double b, const double* __restrict__ y) {
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  for (int k = threadIdx.x; k < sd.K; k += blockDim.x) {
    const int64_t o = sd.voff + k;
    x[o] = a * x[o] + b * y[o];
  }
}

// mode 0: park the active systems assembled in FP64 and factored without a
// shift (their solves need no refinement); mode 1: re-activate the parked ones
__global__ void k_park(int S, int* flags, int mode) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int f = flags[s];
  if (mode == 0) {
    if ((f & F_ACTIVE) && !(f & (F_ASM32 | F_SHIFTED))) flags[s] = (f & ~F_ACTIVE) | F_PARK;
  } else if (f & F_PARK) {
    flags[s] = (f & ~F_PARK) | F_ACTIVE;
  }
}

// Refinement step k of a solve: eta = ||r||_inf / ||rhs||_inf; the system is
// parked (its x final) once accepted, stagnant, or at step kmax.  Slots:
// IRETA (eta of step 0, max over the iteration's solves), IRLAST, IRFAIL,
// IRSTEPS (reset by the iteration's first solve).
__global__ void __launch_bounds__(256) k_ir_check(const SysDesc* __restrict__ sys, int* flags,
                                                  const double* __restrict__ r,
                                                  const double* __restrict__ rhs, double* sc,
                                                  int k, int kmax, int first_solve) {
  __shared__ double sb[256];
  const int s = blockIdx.x;
  ACTIVE_OR_RETURN(s);
  const SysDesc sd = sys[s];
  double rn = 0.0, bn = 0.0;
  for (int i = threadIdx.x; i < sd.K; i += blockDim.x) {
    rn = nanmax(rn, fabs(r[sd.voff + i]));
    bn = nanmax(bn, fabs(rhs[sd.voff + i]));
  }
  rn = wg_max256(rn, sb);
  bn = wg_max256(bn, sb);
  if (threadIdx.x == 0) {
    double eta = bn > 0.0 ? rn / bn : (rn > 0.0 ? INFINITY : 0.0);
    if (!(eta == eta)) eta = INFINITY;
    double* o = sc + (size_t)s * kNSC;
    if (k == 0) {
      if (first_solve) { o[S_IRETA] = eta; o[S_IRFAIL] = 0.0; o[S_IRSTEPS] = 0.0; }
      else o[S_IRETA] = fmax(o[S_IRETA], eta);
    }
    const bool stag = k > 0 && !(eta <= 0.5 * o[S_IRLAST]);
    const bool ok = eta <= kIrTol || (stag && eta <= kIrAccept);
    if (ok || stag || k == kmax) {
      if (!ok) o[S_IRFAIL] = 1.0;
      flags[s] = (flags[s] & ~F_ACTIVE) | F_PARK;
    } else {
      o[S_IRSTEPS] += 1.0;
    }
    o[S_IRLAST] = eta;
  }
}

// Warm start projected into the interior: with W_j = B^T(y)_j - C_j and
// lambda_min(W_j) = cert[2j+1] s_j (bisection on Cholesky),
// Z_j = W_j + tau_j I, tau_j = max(0, theta s_j - lambda_min), and
// X_j = exp(logx_j) I (X_j = I if logx is NULL).
__global__ void k_warm_init(const BlkDesc* __restrict__ blks, const SysDesc* __restrict__ sys,
                            const int* __restrict__ flags, const double* __restrict__ W,
                            const double* __restrict__ cert, const double* __restrict__ logx,
                            double theta, double* X, double* Z) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const double sj = sys[bd.sys].scale[bd.j];
  const double lam = cert[2 * blockIdx.x + 1] * sj;
  const double tau = fmax(0.0, theta * sj - lam);
  const double xs = logx ? exp(logx[blockIdx.x]) : 1.0;
  const int n = bd.n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const bool dg = (e / n) == (e % n);
    Z[bd.off + e] = W[bd.off + e] + (dg ? tau : 0.0);
    X[bd.off + e] = dg ? xs : 0.0;
  }
}

// Centred warm primal: X_j = exp(logx_j) n Zi_j / tr(Zi_j) (Zi = Z^{-1}).
__global__ void k_warm_center(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                              const double* __restrict__ Zi, const double* __restrict__ logx,
                              double* X) {
  __shared__ double tr;
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  const int n = bd.n;
  if (threadIdx.x < 64) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) t += Zi[bd.off + (int64_t)i * n + i];
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
    if (threadIdx.x == 0) tr = t;
  }
  __syncthreads();
  const double f = (logx ? exp(logx[blockIdx.x]) : 1.0) * n / tr;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) X[bd.off + e] = f * Zi[bd.off + e];
}

// out[j] = log(tr(X_j) / n) per block (wave 0 of the workgroup)
__global__ void k_block_logtrace(const BlkDesc* __restrict__ blks, const int* __restrict__ flags,
                                 const double* __restrict__ X, double* out) {
  const BlkDesc bd = blks[blockIdx.x];
  ACTIVE_OR_RETURN(bd.sys);
  double t = 0.0;
  for (int i = threadIdx.x; i < bd.n; i += 64) t += X[bd.off + (int64_t)i * bd.n + i];
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
  if (threadIdx.x == 0) out[blockIdx.x] = log(t / bd.n);
}

// cold start of every block: X = Z = I, C_j = cdiag_j I
__global__ void k_init_blocks(const BlkDesc* __restrict__ blks, const SysDesc* __restrict__ sys,
                              double* X, double* Z, double* Cf) {
  const BlkDesc bd = blks[blockIdx.x];
  const double c = sys[bd.sys].cdiag[bd.j];
  const int n = bd.n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const bool dg = (e / n) == (e % n);
    X[bd.off + e] = dg ? 1.0 : 0.0;
    Z[bd.off + e] = dg ? 1.0 : 0.0;
    Cf[bd.off + e] = dg ? c : 0.0;
  }
}

// launch wrappers ----------------------------------------------------------------

void launch_init_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys, double* X,
                        double* Z, double* Cf) {
  if (nblk) hipLaunchKernelGGL(k_init_blocks, dim3(nblk), dim3(256), 0, st, blks, sys, X, Z, Cf);
}

void launch_warm_init(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                      const int* flags, const double* W, const double* cert, const double* logx,
                      double theta, double* X, double* Z) {
  hipLaunchKernelGGL(k_warm_init, dim3(nblk), dim3(256), 0, st, blks, sys, flags, W, cert, logx, theta,
                     X, Z);
}

void launch_warm_center(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                        const double* Zi, const double* logx, double* X) {
  hipLaunchKernelGGL(k_warm_center, dim3(nblk), dim3(256), 0, st, blks, flags, Zi, logx, X);
}

void launch_block_logtrace(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                           const double* X, double* out) {
  hipLaunchKernelGGL(k_block_logtrace, dim3(nblk), dim3(64), 0, st, blks, flags, X, out);
}

void launch_park(hipStream_t st, int S, int* flags, int mode) {
  hipLaunchKernelGGL(k_park, dim3((S + 255) / 256), dim3(256), 0, st, S, flags, mode);
}

void launch_ir_check(hipStream_t st, int S, const SysDesc* sys, int* flags, const double* r,
                     const double* rhs, double* sc, int k, int kmax, int first_solve) {
  hipLaunchKernelGGL(k_ir_check, dim3(S), dim3(256), 0, st, sys, flags, r, rhs, sc, k, kmax,
                     first_solve);
}

void launch_vec_axpby(hipStream_t st, int S, const SysDesc* sys, const int* flags, double a,
                      double* x, double b, const double* y) {
  hipLaunchKernelGGL(k_vec_axpby, dim3(S), dim3(256), 0, st, sys, flags, a, x, b, y);
}

void launch_pad_identity(hipStream_t st, int S, const SysDesc* sys, double* Lam) {
  hipLaunchKernelGGL(k_pad_identity, dim3(S), dim3(64), 0, st, sys, Lam);
}

static void set_lds(const void* f, size_t bytes) {
  if (bytes > 64 * 1024) hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_cholinv(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                    int* flags, const double* Z, double* Zi) {
  if (nmax_small)
    hipLaunchKernelGGL(k_cholinv16, dim3((nblk + 15) / 16), dim3(256), 0, st, blks, nblk, flags, Z, Zi);
  // orders 64 < n <= 128: the tile factorisation; 16 < n <= 64 (or every
  // order above 16 when some block exceeds 128): the column factorisation in LDS
  const bool tile = maxn > kNB && maxn <= 2 * kNB;
  if (tile) launch_cholinv_tile(st, nblk, blks, flags, Z, Zi);
  if (maxn > kSmallN) {
    const int nmax = tile ? kNB : maxn;
    const size_t lds = (size_t)std::min(maxn, nmax) * std::min(maxn, nmax) * 8;
    set_lds((const void*)k_cholinv, lds);
    hipLaunchKernelGGL(k_cholinv, dim3(nblk), dim3(256), lds, st, blks, flags, Z, Zi, nmax);
  }
}

void launch_ladder(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                   const int* flags, const double* V, const double* dV, double rho, double frac,
                   int len, int* kout) {
  if (nmax_small)
    hipLaunchKernelGGL(k_ladder16, dim3((nblk + 15) / 16), dim3(256), 0, st, blks, nblk, flags, V, dV, rho, frac,
                       len, kout, 1, nullptr, nullptr, nullptr);
  // orders 64 < n <= 128: the tile test; 16 < n <= 64 (or every order above
  // 16 when some block exceeds 128): the column test in LDS
  const bool tile = maxn > kNB && maxn <= 2 * kNB;
  if (tile) launch_ladder_tile(st, nblk, blks, flags, V, dV, rho, frac, len, kout);
  if (maxn > kSmallN) {
    const int nmax = tile ? kNB : maxn;
    const size_t lds = (size_t)std::min(maxn, nmax) * std::min(maxn, nmax) * 8;
    set_lds((const void*)k_ladder, lds);
    hipLaunchKernelGGL(k_ladder, dim3(nblk), dim3(256), lds, st, blks, flags, V, dV, rho, frac, len, kout,
                       nmax);
  }
}

void launch_ladder2(hipStream_t st, int nblk, int maxn, int nmax_small, const BlkDesc* blks,
                    const int* flags, const double* X, const double* dX, const double* Z,
                    const double* dZ, double rho, double frac, int len, int* koutX, int* koutZ) {
  if (nmax_small)
    hipLaunchKernelGGL(k_ladder16, dim3((2 * nblk + 15) / 16), dim3(256), 0, st, blks, nblk, flags, X, dX, rho,
                       frac, len, koutX, 2, Z, dZ, koutZ);
  const bool tile = maxn > kNB && maxn <= 2 * kNB;
  if (tile) {
    launch_ladder_tile(st, nblk, blks, flags, X, dX, rho, frac, len, koutX);
    launch_ladder_tile(st, nblk, blks, flags, Z, dZ, rho, frac, len, koutZ);
  }
  if (maxn > kSmallN) {
    const int nmax = tile ? kNB : maxn;
    const size_t lds = (size_t)std::min(maxn, nmax) * std::min(maxn, nmax) * 8;
    set_lds((const void*)k_ladder, lds);
    hipLaunchKernelGGL(k_ladder, dim3(nblk), dim3(256), lds, st, blks, flags, X, dX, rho, frac, len, koutX,
                       nmax);
    hipLaunchKernelGGL(k_ladder, dim3(nblk), dim3(256), lds, st, blks, flags, Z, dZ, rho, frac, len, koutZ,
                       nmax);
  }
}

void launch_steps_update_y(hipStream_t st, const SysDesc* sys, int S, int maxK, int* flags, const int* koutX,
                           const int* koutZ, double rho, double* sc, double* y, const double* dyh,
                           const double* dyb) {
  const int chunks = std::max(1, (maxK + kYChunk - 1) / kYChunk);
  hipLaunchKernelGGL(k_steps_update_y, dim3((S + 3) / 4, chunks), dim3(256), 0, st, sys, S, flags, koutX, koutZ,
                     rho, sc, y, dyh, dyb);
}

void launch_ladder_step(hipStream_t st, const SysDesc* sys, int S, int* flags, const int* kout,
                        double rho, int slot, double* sc) {
  hipLaunchKernelGGL(k_ladder_step, dim3((S + 3) / 4), dim3(256), 0, st, sys, S, flags, kout, rho, slot, sc);
}

void launch_gemm_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                        const double* sc, const double* A, int tA, const double* B, int tB,
                        double* C, double alpha, int aslot, const double* D, double beta,
                        int bslot, int nmin, int tiles) {
  hipLaunchKernelGGL(k_gemm_blocks, dim3(nblk, tiles), dim3(256), 0, st, blks, flags, sc, A, tA, B, tB, C,
                     alpha, aslot, D, beta, bslot, nmin);
}

void launch_make_G(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                   const double* Cf, const double* S, const double* Z, double* G, int nskip) {
  hipLaunchKernelGGL(k_make_G, dim3(nblk), dim3(256), 0, st, blks, flags, Cf, S, Z, G, nskip);
}

void launch_axpby(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags, double a,
                  const double* A, double b, const double* B, double* out, int nskip) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk), dim3(256), 0, st, blks, flags, a, A, b, B, out, nskip);
}

void launch_symmetrize(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                       const double* W, double* out, int nskip) {
  hipLaunchKernelGGL(k_symmetrize, dim3(nblk), dim3(256), 0, st, blks, flags, W, out, nskip);
}

void launch_combine(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                    const double* dXh, const double* dXb, double* dX, const double* dZh,
                    const double* dZb, double* dZ, int nskip) {
  hipLaunchKernelGGL(k_combine, dim3(nblk), dim3(256), 0, st, blks, flags, dXh, dXb, dX, dZh, dZb, dZ,
                     nskip);
}

void launch_update_blocks(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                          const double* sc, double* X, const double* dX, double* Z,
                          const double* dZ) {
  hipLaunchKernelGGL(k_update_blocks, dim3(nblk), dim3(256), 0, st, blks, flags, sc, X, dX, Z, dZ);
}

void launch_block_red(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags,
                      const double* Cf, const double* X, const double* Z, const double* G,
                      double* red) {
  hipLaunchKernelGGL(k_block_red, dim3(nblk), dim3(256), 0, st, blks, flags, Cf, X, Z, G, red);
}

void launch_sys_finalize(hipStream_t st, int S, const SysDesc* sys, const int* flags,
                         const double* red, const double* y, const double* BX, double sigma,
                         double* sc) {
  hipLaunchKernelGGL(k_sys_finalize, dim3(S), dim3(256), 0, st, sys, flags, red, y, BX, sigma, sc);
}

void launch_form_P(hipStream_t st, int total, const SysDesc* sys, const int* flags,
                   const int* own_pre, int S, const double* y, double* Pm, int nskip) {
  hipLaunchKernelGGL(k_form_P, dim3(total), dim3(256), 0, st, sys, flags, own_pre, S, y, Pm, nskip);
}

void launch_BT_pblk(hipStream_t st, int n, const BlkDesc* pblks, const SysDesc* sys,
                    const int* flags, const double* Pm, double* out, int nskip) {
  if (n) hipLaunchKernelGGL(k_BT_pblk, dim3(n), dim3(256), 0, st, pblks, sys, flags, Pm, out, nskip);
}

void launch_BT_small(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys, const int* flags,
                     const double* y, double* out, const double* Cf, const double* Z, double* G) {
  if (nblk)
    hipLaunchKernelGGL(k_BT_small, dim3((nblk + 3) / 4), dim3(256), 0, st, nblk, blks, sys, flags, y, out,
                       Cf, Z, G);
}

void launch_BT_dblk(hipStream_t st, int n, const BlkDesc* dblks, const SysDesc* sys,
                    const int* flags, const double* Pm, double* out, int nmin, int tiles) {
  if (n) {
    hipLaunchKernelGGL(k_BT_dblk, dim3(n, tiles), dim3(256), 0, st, dblks, sys, flags, Pm, out, nmin);
    hipLaunchKernelGGL(k_BT_dsym, dim3(n), dim3(256), 0, st, dblks, flags, out, nmin);
  }
}

void launch_B_Y(hipStream_t st, int np, const HMPair* pairs, const SysDesc* sys,
                const int* flags, const double* W, double* arena, const BlkDesc* blks, int nmin, int tiles) {
  if (np)
    hipLaunchKernelGGL(k_B_Y, dim3(np, tiles), dim3(256), 0, st, pairs, sys, flags, W, arena, blks, nmin);
}

void launch_B_reduce(hipStream_t st, int totalK, const SysDesc* sys, const int* flags,
                     const int* own_pre, int S, const HMPair* pairs, const double* W,
                     const double* arena, const BlkDesc* blks, double* out, double asub, int nskip) {
  hipLaunchKernelGGL(k_B_reduce, dim3((4 * totalK + 255) / 256), dim3(256), 0, st, sys, flags, own_pre,
                     S, pairs, W, arena, blks, out, asub, nskip);
}

void launch_B_small(hipStream_t st, int totL0, const SysDesc* sys, const int* flags, const int* own_pre,
                    int S, const double* W, double* out, double asub) {
  if (totL0)
    hipLaunchKernelGGL(k_B_small, dim3(totL0), dim3(256), 0, st, sys, flags, own_pre, S, W, out, asub);
}

void launch_pre12(hipStream_t st, int np, const HMPair* pairs, const SysDesc* sys,
                  const int* flags, const double* Zi, const double* X, double* arena,
                  const BlkDesc* blks, const int64_t* offA1, int nmin, int tiles) {
  if (np)
    hipLaunchKernelGGL(k_pre12, dim3(np, tiles), dim3(256), 0, st, pairs, sys, flags, Zi, X, arena, blks,
                       offA1, nmin);
}

void launch_pre34(hipStream_t st, int nq, const HM2* q, const SysDesc* sys, const int* flags,
                  double* arena, int nmin, int tiles) {
  if (nq) hipLaunchKernelGGL(k_pre34, dim3(nq, tiles), dim3(256), 0, st, q, sys, flags, arena, nmin);
}

void launch_certificate(hipStream_t st, int nblk, int maxn, const BlkDesc* blks,
                        const SysDesc* sys, const int* flags, const double* Q, int iters,
                        double* out) {
  hipLaunchKernelGGL(k_certificate16, dim3((nblk + 15) / 16), dim3(256), 0, st, blks, nblk, sys, flags, Q,
                     iters, out);
  const bool tile = maxn > kNB && maxn <= 2 * kNB;
  if (tile) launch_certificate_tile(st, nblk, blks, sys, flags, Q, iters, out);
  if (maxn > kSmallN) {
    const int nmax = tile ? kNB : maxn;
    const size_t lds = (size_t)std::min(maxn, nmax) * std::min(maxn, nmax) * 8;
    set_lds((const void*)k_certificate, lds);
    hipLaunchKernelGGL(k_certificate, dim3(nblk), dim3(256), lds, st, blks, sys, flags, Q, iters, out, nmax);
  }
}

}  // namespace psdp

namespace psdp {

void launch_lift(hipStream_t st, int S, const SysDesc* sys, const int* flags, const double* yin,
                 double* yout) {
  hipLaunchKernelGGL(k_lift, dim3(S), dim3(256), 0, st, sys, flags, yin, yout);
}
void launch_sub_tD(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                   const int* flags, const double* yp, double* out) {
  hipLaunchKernelGGL(k_sub_tD, dim3(nblk), dim3(64), 0, st, blks, sys, flags, yp, out);
}
void launch_B_phase1(hipStream_t st, int S, const SysDesc* sys, const int* flags,
                     const BlkDesc* blks, const double* W, double* out, double asub) {
  hipLaunchKernelGGL(k_B_phase1, dim3(S), dim3(256), 0, st, sys, flags, blks, W, out, asub);
}
void launch_gemm_scaled(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                        const int* flags, const double* A, const double* B, double* C, int tiles) {
  hipLaunchKernelGGL(k_gemm_scaled, dim3(nblk, tiles), dim3(256), 0, st, blks, sys, flags, A, B, C);
}
void launch_lam_phase1(hipStream_t st, int S, int maxK, const SysDesc* sys, const int* flags,
                       const BlkDesc* blks, const double* W, const double* v, double* Lam) {
  hipLaunchKernelGGL(k_lam_phase1_a, dim3(maxK, S), dim3(256), 0, st, sys, flags, Lam);
  hipLaunchKernelGGL(k_lam_phase1_b, dim3(S), dim3(256), 0, st, sys, flags, blks, W, v, Lam);
}
void launch_phase1_vectors(hipStream_t st, int S, const SysDesc* sys, const int* flags, double* yp,
                           double* eK) {
  hipLaunchKernelGGL(k_phase1_vectors, dim3(S), dim3(256), 0, st, sys, flags, yp, eK);
}

}  // namespace psdp

namespace psdp {

// prec = PSDP_PREC_FP32 / _BF16: systems flagged F_ASM32 take that
// reduced-precision kernel, the rest the FP64 one (each kernel skips the
// other's tiles); PSDP_PREC_FP64: the FP64 kernel only.
template <int PR, bool RL, int TPW>
static const void* pair_kernel() {
  if constexpr (PR == 2 || TPW > 7) return (const void*)k_assemble_pair_1wg<PR, RL, TPW>;
  else return (const void*)k_assemble_pair<PR, RL, TPW>;
}

template <int PR>
static void pair_launch(hipStream_t st, int ntiles, int maxn, const AsmTile* tiles,
                        const KTerm* terms, const SysDesc* sys, const int* flags,
                        const double* arena, double* Lam, double* rscr) {
  const int grid = ntiles < kPairGrid ? ntiles : kPairGrid;
  const int n2 = maxn * maxn, NT = (n2 + 15) / 16, n2p = NT * 16;
  const size_t stage = (size_t)2 * kPairKS * n2p * sizeof(typename AsmPrec<PR>::stage_t);
  const size_t rbytes = (size_t)n2 * n2 * 8;
  // R fits LDS next to a second workgroup for n <= 10 (NT <= 7); n = 11
  // (NT = 8) keeps it in global scratch
  const void* f = NT <= 4   ? pair_kernel<PR, true, 2>()
                  : NT <= 6 ? pair_kernel<PR, true, 5>()
                  : NT <= 7 ? pair_kernel<PR, true, 7>()
                            : pair_kernel<PR, false, 8>();
  const size_t lds = NT <= 7 ? (rbytes > stage ? rbytes : stage) : stage;
  set_lds(f, lds);
  int rslot = n2 * n2;
  void* args[] = {(void*)&tiles, (void*)&ntiles, (void*)&terms, (void*)&sys, (void*)&flags,
                  (void*)&arena, (void*)&Lam, (void*)&rscr, (void*)&rslot};
  (void)hipLaunchKernel(f, dim3(grid), dim3(64 * kPairWaves), args, lds, st);
}

void launch_assemble_pair(hipStream_t st, int ntiles, int maxn, const AsmTile* tiles,
                          const KTerm* terms, const SysDesc* sys, const int* flags,
                          const double* arena, double* Lam, int prec, double* rscr) {
  if (!ntiles) return;
  if (prec == PSDP_PREC_FP32) pair_launch<1>(st, ntiles, maxn, tiles, terms, sys, flags, arena, Lam, rscr);
  if (prec == PSDP_PREC_BF16) pair_launch<2>(st, ntiles, maxn, tiles, terms, sys, flags, arena, Lam, rscr);
  pair_launch<0>(st, ntiles, maxn, tiles, terms, sys, flags, arena, Lam, rscr);
}

void launch_assemble_grp(hipStream_t st, int ntiles, const AsmTile* tiles, const KTerm* terms,
                         const SysDesc* sys, const int* flags, const int* gpinfo,
                         const double* arena, double* Lam, const int64_t* gpoff, int prec) {
  if (!ntiles) return;
  if (prec == PSDP_PREC_FP32)
    hipLaunchKernelGGL(k_assemble_grp<1>, dim3(ntiles), dim3(64 * kGrpW), 0, st, tiles, terms, sys, flags,
                       gpinfo, arena, Lam, gpoff);
  if (prec == PSDP_PREC_BF16)
    hipLaunchKernelGGL(k_assemble_grp<2>, dim3(ntiles), dim3(64 * kGrpW), 0, st, tiles, terms, sys, flags,
                       gpinfo, arena, Lam, gpoff);
  hipLaunchKernelGGL(k_assemble_grp<0>, dim3(ntiles), dim3(64 * kGrpW), 0, st, tiles, terms, sys, flags,
                     gpinfo, arena, Lam, gpoff);
}

}  // namespace psdp

namespace psdp {

static int small_G(int nmax) { return nmax >= 1 && nmax <= kSmallN ? 256 / (nmax * nmax) : 0; }

bool use_small(int nmax) { return small_G(nmax) > 0; }

void launch_sym_ZAX_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                          const double* Zi, const double* A, const double* X, double* W1) {
  const int G = small_G(nmax);
  hipLaunchKernelGGL(k_sym_ZAX_small, dim3((nblk + G - 1) / G), dim3(256), 0, st, nblk, nmax, G, blks,
                     flags, Zi, A, X, W1);
}

void launch_pred_dir_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                           const double* sc, const double* S1, const double* Gm, const double* Zi,
                           const double* X, double* dZh, double* dXh, double* Wc, double* W1) {
  const int G = small_G(nmax);
  hipLaunchKernelGGL(k_pred_dir_small, dim3((nblk + G - 1) / G), dim3(256), 0, st, nblk, nmax, G, blks,
                     flags, sc, S1, Gm, Zi, X, dZh, dXh, Wc, W1);
}

void launch_corr_dir_small(hipStream_t st, int nblk, int nmax, const BlkDesc* blks, const int* flags,
                           const double* Zi, const double* dZb, const double* X, const double* Wc,
                           const double* dXh, const double* dZh, double* dX, double* dZ) {
  const int G = small_G(nmax);
  hipLaunchKernelGGL(k_corr_dir_small, dim3((nblk + G - 1) / G), dim3(256), 0, st, nblk, nmax, G, blks,
                     flags, Zi, dZb, X, Wc, dXh, dZh, dX, dZ);
}

void launch_pre12_small(hipStream_t st, int np, int nmax, const HMPair* pairs, const SysDesc* sys,
                        const int* flags, const double* Zi, const double* X, double* arena,
                        const BlkDesc* blks, const int64_t* offA1) {
  const int G = small_G(nmax);
  if (np) hipLaunchKernelGGL(k_pre12_small, dim3((np + G - 1) / G), dim3(256), 0, st, np, nmax, G, pairs, sys, flags, Zi, X, arena, blks, offA1);
}

void launch_pre34_small(hipStream_t st, int nq, int nmax, const HM2* q, const SysDesc* sys,
                        const int* flags, double* arena) {
  const int G = small_G(nmax);
  if (nq) hipLaunchKernelGGL(k_pre34_small, dim3((nq + G - 1) / G), dim3(256), 0, st, nq, nmax, G, q, sys, flags, arena);
}

}  // namespace psdp
