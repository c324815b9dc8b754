// Dense FP64 Cholesky of the Schur complement and the two triangular solves
// (Alg. 2, root steps 1 and 2: Lambda dy = Omega).  The paper factors Lambda
// on a root processor with LAPACK; here every system of a batch is factored
// together, tile by tile.
//
// Storage: each system's Kpad x Kpad matrix is row-major (leading dimension
// Kpad, a multiple of 64); rows/columns past K hold the identity, so the
// factor of the padded matrix is blockdiag(L, I) and no kernel needs ragged
// edges.  The off-diagonal tiles of the factor overwrite the lower triangle;
// the factored diagonal tiles L_pp and their inverses go to separate arrays
// (other workgroups of the same step still read the unfactored diagonal
// tile); the strict upper triangle keeps Lambda.
//
// Right-looking blocked algorithm, step p (panel column p):
//   diag   : one workgroup per system factors the 64 x 64 diagonal tile in
//            registers and inverts the factor (L_pp, L_pp^{-1} stored);
//   trsm   : one workgroup per tile row i > p forms L_ip = A_ip L_pp^{-T};
//   update : two levels.  Panels are grouped in super-panels of kSW; inside
//            one, each tile (i, j) with p < j <= (end of the super-panel)
//            gets A_ij -= L_ip L_jp^T right away (narrow update, depth 64);
//            after the super-panel's last panel, every tile right of it gets
//            the super-panel's whole contribution in one pass of depth
//            64 kSW (wide update).  Both on FP64 MFMA.
// Steps are launched for the whole batch; a (step, system) table maps
// workgroups to systems.  Triangular solves use the stored inverses, so the
// diagonal solves are matrix-vector products.
#include <hip/hip_runtime.h>

#include "devcommon.h"
#include "internal.h"

namespace psdp {

constexpr int LDT = kNB + 1;   // LDS leading dimension of a 64 x 64 tile
typedef double v4d __attribute__((ext_vector_type(4)));

// Register-resident factorisation of a 64 x 64 tile with 256 threads: thread
// (tr, tc) owns rows tr + 16a and columns tc + 16b (a, b < 4).  Column k is
// broadcast through a double-buffered LDS vector, so each column costs one
// barrier and eight LDS reads per thread.  Non-positive or non-finite pivots
// set *fail and are replaced by 1.  On return reg holds L (lower part).
__device__ inline void reg_potrf64(double (&reg)[4][4], double* colbuf /*2 x 64*/, int* fail) {
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  // publish column 0
  if (tc == 0)
#pragma unroll
    for (int a = 0; a < 4; ++a) colbuf[tr + 16 * a] = reg[a][0];
  for (int k = 0; k < kNB; ++k) {
    __syncthreads();
    const double* cb = colbuf + (k & 1) * kNB;
    double d = cb[k];
    const bool bad = !(d > 0.0) || !isfinite(d);
    d = bad ? 1.0 : d;
    const double piv = sqrt(d);
    const double rpiv = 1.0 / piv;   // one reciprocal per column, then products
    if (bad && tid == 0) *fail = 1;
    double li[4], lj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) li[a] = cb[tr + 16 * a] * rpiv;
#pragma unroll
    for (int b = 0; b < 4; ++b) lj[b] = cb[tc + 16 * b] * rpiv;
    // branch-free update of the owned 4 x 4 block
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = tr + 16 * a;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = tc + 16 * b;
        const double upd = reg[a][b] - li[a] * lj[b];
        const double colk = i > k ? li[a] : (i == k ? piv : reg[a][b]);
        reg[a][b] = j == k ? colk : ((j > k && j <= i) ? upd : reg[a][b]);
      }
    }
    // publish column k+1 (final: all updates through column k applied)
    const int kn = k + 1;
    if (kn < kNB && tc == (kn & 15)) {
      const int bs = kn >> 4;
      double* nb = colbuf + (kn & 1) * kNB;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double v = bs == 0 ? reg[a][0] : bs == 1 ? reg[a][1] : bs == 2 ? reg[a][2] : reg[a][3];
        nb[tr + 16 * a] = v;
      }
    }
  }
  __syncthreads();
}

// X = L^{-1} by forward substitution on the identity, register-resident in the
// same 4 x 4 ownership: step k scales row k of X by 1/L[k][k] (reciprocals
// of the diagonal precomputed) and removes L[i][k] X[k][:] from every row
// i > k.  L is read from LDS (leading dimension LDT), row k of X is broadcast
// through a double-buffered LDS vector.
__device__ inline void reg_trinv64(const double* sL, double (&X)[4][4], double* rowbuf,
                                   double* rdiag) {
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  if (tid < kNB) rdiag[tid] = 1.0 / sL[tid * LDT + tid];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) X[a][b] = (tr + 16 * a == tc + 16 * b) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = 0; k < kNB; ++k) {
    double* rb = rowbuf + (k & 1) * kNB;
    const double rkk = rdiag[k];
    // the owners of row k scale it and publish it
    if (tr == (k & 15)) {
      const int as = k >> 4;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) X[a][b] = a == as ? X[a][b] * rkk : X[a][b];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double v = as == 0 ? X[0][b] : as == 1 ? X[1][b] : as == 2 ? X[2][b] : X[3][b];
        rb[tc + 16 * b] = v;
      }
    }
    __syncthreads();
    double xk[4], lik[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) xk[b] = rb[tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a) lik[a] = sL[(tr + 16 * a) * LDT + k];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (tr + 16 * a > k)
#pragma unroll
        for (int b = 0; b < 4; ++b) X[a][b] -= lik[a] * xk[b];
  }
  __syncthreads();
}

// Diagonal step p: one workgroup per system factors the 64 x 64 tile A_pp
// and inverts the factor, storing L_pp and L_pp^{-1}.
__global__ void __launch_bounds__(256) k_chol_diag(const SysDesc* __restrict__ sys, int* flags,
                                                   const double* __restrict__ Lam, double* Ldiag,
                                                   double* Linv, const int* __restrict__ st_sys,
                                                   int p) {
  __shared__ double sL[kNB * LDT];
  __shared__ double vbuf[2 * kNB];
  __shared__ double rdiag[kNB];
  __shared__ int fl;
  const int s = st_sys[blockIdx.x];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  const double* A = Lam + sd.loff;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  if (tid == 0) fl = 0;
  const double* App = A + (int64_t)p * kNB * ld + (int64_t)p * kNB;
  double reg[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) reg[a][b] = App[(int64_t)(tr + 16 * a) * ld + tc + 16 * b];
  reg_potrf64(reg, vbuf, &fl);
  double* D = Ldiag + sd.dgoff + (int64_t)p * kNB * kNB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = tr + 16 * a, j = tc + 16 * b;
      const double v = j <= i ? reg[a][b] : 0.0;
      sL[i * LDT + j] = v;
      D[i * kNB + j] = v;
    }
  __syncthreads();
  double X[4][4];
  reg_trinv64(sL, X, vbuf, rdiag);
  double* Dv = Linv + sd.dgoff + (int64_t)p * kNB * kNB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Dv[(tr + 16 * a) * kNB + tc + 16 * b] = X[a][b];
  if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
}

// Panel step p: L_ip = A_ip L_pp^{-T} for every tile row i > p, on FP64
// MFMA (C[r][c] = sum_k A_ip[r][k] X[c][k] with X = L_pp^{-1}).
__global__ void __launch_bounds__(256) k_chol_trsm(const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ flags, double* Lam,
                                                   const double* __restrict__ Linv,
                                                   const int* __restrict__ st_sys,
                                                   const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sA[kNB * LDT];
  __shared__ double sX[kNB * LDT];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  const int i = p + 1 + t;
  double* Ai = Lam + sd.loff + (int64_t)i * kNB * ld + (int64_t)p * kNB;
  const double* Xg = Linv + sd.dgoff + (int64_t)p * kNB * kNB;
  const int tid = threadIdx.x;
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e >> 6, c = e & 63;
    sA[r * LDT + c] = Ai[(int64_t)r * ld + c];
    sX[r * LDT + c] = Xg[e];
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < kNB; k0 += 4) {
    const double av = sA[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double bv = sX[(16 * u + r16) * LDT + k0 + kq];
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) Ai[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16] = acc[u][q];
}

// Narrow update (inside the super-panel of p): A_ij -= L_ip L_jp^T for the
// columns p < j <= end of the super-panel and every row i >= j, on FP64 MFMA: wave w owns
// rows 16w..16w+15 and the four 16-column tiles; both panels staged in LDS.
__global__ void __launch_bounds__(256) k_chol_update(const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags, double* Lam,
                                                     const int* __restrict__ st_sys,
                                                     const int* __restrict__ st_pre, int cnt,
                                                     int p) {
  __shared__ double sa[kNB * LDT];
  __shared__ double sb[kNB * LDT];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  // column j = p + 1 + c (c < number of super-panel columns right of p),
  // rows i = j .. P-1: column c holds R - c tiles, R = P - p - 1
  const int R = sd.P - p - 1;
  int c = 0, base = 0;
  while (t >= base + (R - c)) { base += R - c; ++c; }
  const int j = p + 1 + c, i = j + (t - base);
  const double* Li = A + (int64_t)i * kNB * ld + (int64_t)p * kNB;
  const double* Lj = A + (int64_t)j * kNB * ld + (int64_t)p * kNB;
  double* C = A + (int64_t)i * kNB * ld + (int64_t)j * kNB;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e >> 6, c = e & 63;
    sa[r * LDT + c] = Li[(int64_t)r * ld + c];
    sb[r * LDT + c] = Lj[(int64_t)r * ld + c];
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
  const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < kNB; k0 += 4) {
    const double a = sa[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double b = sb[(16 * u + r16) * LDT + k0 + kq];
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cc = 16 * u + r16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = 16 * w + 4 * q + kq;
      if (i != j || cc <= rr) C[(int64_t)rr * ld + cc] -= acc[u][q];
    }
  }
}

// Wide update at the end of a super-panel of kSW panels (p = its last
// panel): A_ij -= sum over the super-panel's panels q of L_iq L_jq^T for every
// tile pair right of it (depth 64 kSW), on 128 x 128 output blocks (2 x 2
// tiles; wave w owns the 64 x 64 quadrant (w/2, w%2) as 4 x 4 MFMA tiles).
// The depth is staged through LDS 16 columns at a time with the next chunk
// prefetched into registers.  Only the lower triangle (column <= row) of the
// matrix is written; rows or columns past Kpad are skipped.
constexpr int kWT = 128, kWK = 16, kWLD = kWK + 1;

__global__ void __launch_bounds__(256) k_chol_update_wide(const SysDesc* __restrict__ sys,
                                                          const int* __restrict__ flags, double* Lam,
                                                          const int* __restrict__ st_sys,
                                                          const int* __restrict__ st_pre, int cnt,
                                                          int p) {
  __shared__ double sa[kWT * kWLD];
  __shared__ double sb[kWT * kWLD];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const int q0 = p + 1;
  const int r0 = kNB * (q0 + 2 * bi), c0 = kNB * (q0 + 2 * bj);
  const int nmax = sd.Kpad;
  const int d0 = kNB * (p - kSW + 1), D = kNB * kSW;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // staging map: thread loads rows (tid / 16) + 16 u, column tid % 16
  const int lr = tid >> 4, lk = tid & 15;
  double ra[8], rb[8];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = lr + 16 * u;
      ra[u] = r0 + row < nmax ? A[(int64_t)(r0 + row) * ld + d0 + kc + lk] : 0.0;
      rb[u] = c0 + row < nmax ? A[(int64_t)(c0 + row) * ld + d0 + kc + lk] : 0.0;
    }
  };
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int kc = 0; kc < D; kc += kWK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sa[(lr + 16 * u) * kWLD + lk] = ra[u];
      sb[(lr + 16 * u) * kWLD + lk] = rb[u];
    }
    __syncthreads();
    if (kc + kWK < D) load(kc + kWK);
#pragma unroll
    for (int ks = 0; ks < kWK; ks += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sa[(wr + 16 * a + r16) * kWLD + ks + kq];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sb[(wc + 16 * b + r16) * kWLD + ks + kq];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int R = r0 + wr + 16 * a + 4 * q + kq;
        const int Cc = c0 + wc + 16 * b + r16;
        if (R < nmax && Cc < nmax && Cc <= R) A[(int64_t)R * ld + Cc] -= acc[a][b][q];
      }
}

// y = M x or M^T x for a 64 x 64 tile M in global memory (row-major, leading
// dimension ldm) and x in LDS; four lanes per output row; result in LDS.
__device__ inline void tile_mv64(const double* M, int64_t ldm, bool trans, const double* x,
                                 double* y) {
  const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
  double part = 0.0;
  if (!trans) {
    for (int c = q; c < kNB; c += 4) part += M[(int64_t)row * ldm + c] * x[c];
  } else {
    for (int c = q; c < kNB; c += 4) part += M[(int64_t)c * ldm + row] * x[c];
  }
  part += __shfl_xor(part, 1, 4);
  part += __shfl_xor(part, 2, 4);
  if (q == 0) y[row] = part;
}

// forward step p: z_p = L_pp^{-1} r_p (tile 0 writes it); tiles i > p update
// r_i -= L_ip z_p.
__global__ void __launch_bounds__(256) k_trsv_fwd(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ Lam,
                                                  const double* __restrict__ Linv, double* r,
                                                  double* z, const int* __restrict__ st_sys,
                                                  const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sx[kNB], sz[kNB];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* rs = r + sd.voff;
  double* zs = z + sd.voff;
  if (threadIdx.x < kNB) sx[threadIdx.x] = rs[p * kNB + threadIdx.x];
  __syncthreads();
  tile_mv64(Linv + sd.dgoff + (int64_t)p * kNB * kNB, kNB, false, sx, sz);
  __syncthreads();
  if (t == 0) {
    if (threadIdx.x < kNB) zs[p * kNB + threadIdx.x] = sz[threadIdx.x];
    return;
  }
  const int i = p + t;
  tile_mv64(Lam + sd.loff + (int64_t)i * kNB * ld + (int64_t)p * kNB, ld, false, sz, sx);
  __syncthreads();
  if (threadIdx.x < kNB) rs[i * kNB + threadIdx.x] -= sx[threadIdx.x];
}

// backward step p: x_p = L_pp^{-T} z_p (tile p writes it); tiles i < p
// update z_i -= L_pi^T x_p.
__global__ void __launch_bounds__(256) k_trsv_bwd(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ Lam,
                                                  const double* __restrict__ Linv, double* z,
                                                  double* x, const int* __restrict__ st_sys,
                                                  const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sx[kNB], sz[kNB];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int i = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* zs = z + sd.voff;
  double* xs = x + sd.voff;
  if (threadIdx.x < kNB) sz[threadIdx.x] = zs[p * kNB + threadIdx.x];
  __syncthreads();
  tile_mv64(Linv + sd.dgoff + (int64_t)p * kNB * kNB, kNB, true, sz, sx);
  __syncthreads();
  if (i == p) {
    if (threadIdx.x < kNB) xs[p * kNB + threadIdx.x] = sx[threadIdx.x];
    return;
  }
  tile_mv64(Lam + sd.loff + (int64_t)p * kNB * ld + (int64_t)i * kNB, ld, true, sx, sz);
  __syncthreads();
  if (threadIdx.x < kNB) zs[i * kNB + threadIdx.x] -= sz[threadIdx.x];
}

// Whole solve L L^T x = rhs for systems with few tiles: one workgroup per
// system sweeps all tile steps (no inter-workgroup dependency).  r is
// scratch; x receives the solution.
__global__ void __launch_bounds__(256) k_trsv_small(const SysDesc* __restrict__ sys,
                                                    const int* __restrict__ flags,
                                                    const int* __restrict__ small_ids,
                                                    const double* __restrict__ Lam,
                                                    const double* __restrict__ Linv,
                                                    const double* __restrict__ rhs, double* r,
                                                    double* x) {
  __shared__ double sv[kNB], sw[kNB];
  const int s = small_ids[blockIdx.x];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  const double* A = Lam + sd.loff;
  const double* Di = Linv + sd.dgoff;
  double* rs = r + sd.voff;
  double* xs = x + sd.voff;
  const int tid = threadIdx.x;
  for (int k = tid; k < sd.Kpad; k += 256) rs[k] = rhs[sd.voff + k];
  __syncthreads();
  // forward: z_p = L_pp^{-1} r_p, r_i -= L_ip z_p (z kept in r)
  for (int p = 0; p < sd.P; ++p) {
    if (tid < kNB) sv[tid] = rs[p * kNB + tid];
    __syncthreads();
    tile_mv64(Di + (int64_t)p * kNB * kNB, kNB, false, sv, sw);
    __syncthreads();
    if (tid < kNB) rs[p * kNB + tid] = sw[tid];
    const int rows = (sd.P - p - 1) * kNB;
    for (int rr = tid; rr < rows; rr += 256) {
      const double* Lrow = A + (int64_t)((p + 1) * kNB + rr) * ld + (int64_t)p * kNB;
      double acc = 0.0;
      for (int c = 0; c < kNB; ++c) acc += Lrow[c] * sw[c];
      rs[(p + 1) * kNB + rr] -= acc;
    }
    __syncthreads();
  }
  // backward: x_p = L_pp^{-T} z_p, z_i -= L_pi^T x_p
  for (int p = sd.P - 1; p >= 0; --p) {
    if (tid < kNB) sv[tid] = rs[p * kNB + tid];
    __syncthreads();
    tile_mv64(Di + (int64_t)p * kNB * kNB, kNB, true, sv, sw);
    __syncthreads();
    if (tid < kNB) xs[p * kNB + tid] = sw[tid];
    const int cols = p * kNB;
    for (int cc = tid; cc < cols; cc += 256) {
      double acc = 0.0;
      for (int c = 0; c < kNB; ++c) acc += A[(int64_t)(p * kNB + c) * ld + cc] * sw[c];
      rs[cc] -= acc;
    }
    __syncthreads();
  }
}

// launch wrappers --------------------------------------------------------------

void launch_chol_diag(hipStream_t st, const SysDesc* sys, int* flags, const double* Lam,
                      double* Ldiag, double* Linv, const int* ssys, int cnt, int p) {
  if (cnt)
    hipLaunchKernelGGL(k_chol_diag, dim3(cnt), dim3(256), 0, st, sys, flags, Lam, Ldiag, Linv, ssys, p);
}

void launch_chol_trsm(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                      const double* Linv, const int* ssys, const int* spre, int cnt, int total,
                      int p) {
  if (total)
    hipLaunchKernelGGL(k_chol_trsm, dim3(total), dim3(256), 0, st, sys, flags, Lam, Linv, ssys, spre,
                       cnt, p);
}

void launch_chol_update(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                        const int* ssys, const int* spre, int cnt, int total, int p) {
  hipLaunchKernelGGL(k_chol_update, dim3(total), dim3(256), 0, st, sys, flags, Lam, ssys, spre, cnt, p);
}

void launch_chol_update_wide(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                             const int* ssys, const int* spre, int cnt, int total, int p) {
  if (total)
    hipLaunchKernelGGL(k_chol_update_wide, dim3(total), dim3(256), 0, st, sys, flags, Lam, ssys, spre,
                       cnt, p);
}

void launch_trsv_fwd(hipStream_t st, const SysDesc* sys, const int* flags, const double* Lam,
                     const double* Linv, double* r, double* z, const int* ssys, const int* spre,
                     int cnt, int total, int p) {
  hipLaunchKernelGGL(k_trsv_fwd, dim3(total), dim3(256), 0, st, sys, flags, Lam, Linv, r, z, ssys, spre, cnt, p);
}

void launch_trsv_bwd(hipStream_t st, const SysDesc* sys, const int* flags, const double* Lam,
                     const double* Linv, double* z, double* x, const int* ssys, const int* spre,
                     int cnt, int total, int p) {
  hipLaunchKernelGGL(k_trsv_bwd, dim3(total), dim3(256), 0, st, sys, flags, Lam, Linv, z, x, ssys, spre, cnt, p);
}

void launch_trsv_small(hipStream_t st, int nsmall, const SysDesc* sys, const int* flags,
                       const int* small_ids, const double* Lam, const double* Linv,
                       const double* rhs, double* r, double* x) {
  if (nsmall)
    hipLaunchKernelGGL(k_trsv_small, dim3(nsmall), dim3(256), 0, st, sys, flags, small_ids, Lam, Linv,
                       rhs, r, x);
}

}  // namespace psdp
