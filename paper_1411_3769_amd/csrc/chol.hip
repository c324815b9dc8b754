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
//   diag   : one workgroup per system factors the 64 x 64 diagonal tile and
//            inverts the factor (L_pp, L_pp^{-1} stored);
//   trsm   : one workgroup per tile row i > p forms L_ip = A_ip L_pp^{-T};
//   update : two levels.  Panels are grouped in super-panels of sw (the
//            last one absorbs a shorter remainder); inside one, each tile
//            (i, j) with p < j <= (end of the super-panel) gets
//            A_ij -= L_ip L_jp^T right away (narrow update, depth 64), and
//            the workgroup of tile (p+1, p+1) goes on to the diagonal step
//            of p + 1; after the super-panel's last panel, every tile right
//            of it gets the super-panel's whole contribution in one pass of
//            depth 64 sw (wide update).  Both on FP64 MFMA.  sw is chosen
//            per system (the autotuner times 4, 8 and 16).
// Left-looking alternative (k_chol_left, below 64 tiles when the autotuner
// finds it faster): one launch per tile column; each tile gathers its whole
// update from the finished columns and is written once.
// Steps are launched for the whole batch; a (step, system) table maps
// workgroups to systems.  Triangular solves use the stored inverses, so the
// diagonal solves are matrix-vector products.
#include <hip/hip_runtime.h>

#include "devcommon.h"
#include "internal.h"

namespace psdp {

constexpr int LDT = kNB + 1;   // LDS leading dimension of a 64 x 64 tile
typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Diagonal tile: blocked factorisation and inverse of a 64 x 64 tile by one
// workgroup.  The tile is split in 4 x 4 blocks of 16 x 16.  For each block
// column kb: wave 0 factors the diagonal block in registers and inverts its
// factor (wave-wide shuffles, no barriers), the other waves form the blocks
// below it on MFMA (L_ik = A_ik X_kk^T) and update the trailing blocks
// (A_ij -= L_ik L_jk^T).  The inverse's off-diagonal blocks then follow by
// block forward substitution, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj.
// ---------------------------------------------------------------------------
constexpr int kLD = 65;          // LDS leading dimension of the 64 x 64 tiles
constexpr int kBL = 16;          // block order

// 16 x 16 x 16 product on FP64 MFMA for one wave: acc += P Q (qt = false) or
// P Q^T (qt = true); P, Q in LDS with leading dimension ld.
__device__ inline v4d mm16(const double* P, const double* Q, bool qt, v4d acc) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const double a = P[r16 * kLD + 4 * ks + kq];
    const double b = qt ? Q[r16 * kLD + 4 * ks + kq] : Q[(4 * ks + kq) * kLD + r16];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// store (sign * acc) or add it (accumulate) into a 16 x 16 block in LDS
__device__ inline void st16(double* D, v4d acc, double sign, bool add) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double* d = D + (4 * i + kq) * kLD + r16;
    *d = add ? *d + sign * acc[i] : sign * acc[i];
  }
}

// Wave-level factorisation and inverse of the 16 x 16 block at B (leading
// dimension kLD; lower triangle read).  Lane r of each 16-lane row of the
// wave holds row r of A (a[]) and column r of X = L^{-1} (x[]); the four
// rows of the wave compute the same block and the first writes it.  Step k:
// column k of L is the pivot's column scaled by the Newton reciprocal
// square root of the pivot, x_k = b_k / L_kk, and every later c gets
// a_c -= L_rk L_ck and b_c -= L_ck x_k (the forward substitution for X
// carried along with the factorisation, b starting as the unit vector
// e_r).  L_ck reaches every lane by a DPP row broadcast from lane c, so no
// value goes through LDS.  Above the diagonal a[] collects values nothing
// reads; the store writes zeros there.  On return B holds L (zeros above
// the diagonal) and Xb holds L^{-1}.  Non-positive pivots set *fail
// (replaced by 1).
__device__ inline void wave_potri16(double* B, double* Xb, int* fail) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  double a[16], x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = c <= r ? B[r * kLD + c] : 0.0;
    x[c] = c == r ? 1.0 : 0.0;
  }
  bool bad = false;
  static_for<16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double d = row_bcast16<k>(a[k]);
    const bool bb = !(d > 0.0) || !isfinite(d);
    bad = bad || bb;
    d = bb ? 1.0 : d;
    const double rs = rsqrt_nr(d);
    const double lrk = r > k ? a[k] * rs : (r == k ? d * rs : 0.0);
    a[k] = lrk;
    x[k] *= rs;
    static_for<16>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c > k) {
        const double lck = row_bcast16<c>(lrk);
        a[c] -= lrk * lck;
        x[c] -= lck * x[k];
        // x_c is final for this step here: left to itself the compiler
        // sinks the x updates past the whole factorisation and keeps every
        // broadcast L_ck alive until then (hundreds of registers)
        asm volatile("" : "+v"(x[c]));
      }
    });
  });
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      B[r * kLD + c] = c <= r ? a[c] : 0.0;
      Xb[c * kLD + r] = x[c];
    }
  }
  if (bad && lane == 0) *fail = 1;
}

// Factorisation and inverse of the 64 x 64 tile in sA (lower triangle read)
// by the 4 waves of a workgroup: on return sA holds L_pp (lower triangle) and
// sX (zero on entry) holds L_pp^{-1}.  The strictly upper blocks of sA serve
// as scratch for the inverse.  Non-positive pivots set *fl.
__device__ __forceinline__ void diag_tile(double* sA, double* sX, int* fl) {
  const int w = threadIdx.x >> 6;
  auto blk = [](double* M, int i, int j) { return M + (kBL * i) * kLD + kBL * j; };
  for (int kb = 0; kb < 4; ++kb) {
    if (w == 0) wave_potri16(blk(sA, kb, kb), blk(sX, kb, kb), fl);
    __syncthreads();
    // L_ik = A_ik X_kk^T for the blocks below (wave w takes i = kb + w); the
    // result overwrites A_ik after a barrier
    const bool trs = w >= 1 && kb + w < 4;
    v4d tacc = v4d{0.0, 0.0, 0.0, 0.0};
    if (trs) tacc = mm16(blk(sA, kb + w, kb), blk(sX, kb, kb), true, tacc);
    __syncthreads();
    if (trs) st16(blk(sA, kb + w, kb), tacc, 1.0, false);
    __syncthreads();
    // A_ij -= L_ik L_jk^T for kb < j <= i
    int t = 0;
    for (int i = kb + 1; i < 4; ++i)
      for (int j = kb + 1; j <= i; ++j, ++t) {
        if ((t & 3) != w) continue;
        v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
        acc = mm16(blk(sA, i, kb), blk(sA, j, kb), true, acc);
        st16(blk(sA, i, j), acc, -1.0, true);
      }
    __syncthreads();
  }
  // off-diagonal blocks of X, by distance d = i - j
  for (int dd = 1; dd < 4; ++dd) {
    // T = sum_{k=j}^{i-1} L_ik X_kj, wave w takes j = w; T goes to the upper
    // block (0, w + 1) of sA
    const int j = w, i = w + dd;
    double* T = blk(sA, 0, w + 1);
    if (i < 4) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; ++k) acc = mm16(blk(sA, i, k), blk(sX, k, j), false, acc);
      st16(T, acc, 1.0, false);
    }
    __syncthreads();
    if (i < 4) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      acc = mm16(blk(sX, i, i), T, false, acc);
      st16(blk(sX, i, j), acc, -1.0, false);
    }
    __syncthreads();
  }
}

// store the lower triangles of sA (L_pp) and sX (L_pp^{-1}) as dense tiles
__device__ inline void store_diag(const double* sA, const double* sX, double* D, double* Dv) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    const int r = e >> 6, cc = e & 63;
    D[e] = cc <= r ? sA[r * kLD + cc] : 0.0;
    Dv[e] = cc <= r ? sX[r * kLD + cc] : 0.0;
  }
}

// Cholesky test of the 128 x 128 matrix [[A11, A21^T], [A21, A22]] held in
// sA (A11), sB (A21) and sC (A22) by the tile routine: diag_tile on A11,
// L21 = A21 L11^{-T} and A22 - L21 L21^T on MFMA, diag_tile on that; a
// non-positive pivot anywhere sets *fl.  sX is scratch; the four tiles are
// overwritten.  Entered and left with every thread past a barrier.
__device__ __forceinline__ void tile_chol_test(double* sA, double* sX, double* sB, double* sC, int* fl) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  // acc = X Y^T for 64 x 64 tiles in LDS (wave w: rows 16w..16w+15)
  auto prodT = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * kLD + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double b = Y[(16 * u + r16) * kLD + k0 + kq];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  };
  for (int e = tid; e < kNB * kNB; e += 256) sX[(e >> 6) * kLD + (e & 63)] = 0.0;
  __syncthreads();
  diag_tile(sA, sX, fl);
  __syncthreads();
  v4d acc[4] = {};
  prodT(sB, sX, acc);   // L_21 = A_21 L_11^{-T}
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sB[(16 * w + 4 * q + kq) * kLD + 16 * u + r16] = acc[u][q];
  __syncthreads();
  v4d upd[4] = {};
  prodT(sB, sB, upd);   // L_21 L_21^T
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sC[(16 * w + 4 * q + kq) * kLD + 16 * u + r16] -= upd[u][q];
  for (int e = tid; e < kNB * kNB; e += 256) sX[(e >> 6) * kLD + (e & 63)] = 0.0;
  __syncthreads();
  diag_tile(sC, sX, fl);
  __syncthreads();
}

// Step-length ladder for blocks of order 64 < n <= 128 (the reading of the
// paper's line search that keeps X and Z positive definite): r_0 = 1,
// r_{k+1} = rho r_k; block b records the first k at which V_b + (r_k / frac)
// dV_b passes Cholesky, -1 if none up to len.  The trial matrix (formed with
// a separate multiply and add) is padded with the identity to 128 and
// tested with the Schur Cholesky's blocked tile factorisation: diag_tile on
// A_11, then L_21 = A_21 L_11^{-T} and A_22 - L_21 L_21^T on MFMA, and
// diag_tile on that (a non-positive pivot anywhere fails the rung).  Smaller
// orders keep the column-by-column test, which is faster there.
__global__ void __launch_bounds__(256) k_ladder_tile(const BlkDesc* __restrict__ blks,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ V,
                                                     const double* __restrict__ dV, double rho,
                                                     double frac, int len, int* kout) {
  __shared__ double sA[kNB * kLD];   // A_11, then L_11
  __shared__ double sX[kNB * kLD];   // L_11^{-1} (zero before each diag_tile)
  __shared__ double sB[kNB * kLD];   // A_21, then L_21
  __shared__ double sC[kNB * kLD];   // A_22
  __shared__ int fl;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kNB || bd.n > 2 * kNB) return;   // k_ladder16 / k_ladder
  const int tid = threadIdx.x;
  if (!(flags[bd.sys] & F_ACTIVE)) {
    if (tid == 0) kout[blockIdx.x] = 0;
    return;
  }
  const int n = bd.n;
  const double* Vb = V + bd.off;
  const double* dVb = dV + bd.off;
  // entry (i, j) of the padded trial matrix
  auto trial = [&](int i, int j, double t) {
    if (i < n && j < n) return __dadd_rn(Vb[i * n + j], __dmul_rn(t, dVb[i * n + j]));
    return i == j ? 1.0 : 0.0;
  };
  double r = 1.0;
  int found = -1;
  for (int k = 0; k <= len; ++k) {
    const double t = r / frac;
    for (int e = tid; e < kNB * kNB; e += 256) {
      const int i = e >> 6, j = e & 63;
      sA[i * kLD + j] = trial(i, j, t);
      sB[i * kLD + j] = trial(kNB + i, j, t);
      sC[i * kLD + j] = trial(kNB + i, kNB + j, t);
    }
    if (tid == 0) fl = 0;
    tile_chol_test(sA, sX, sB, sC, &fl);
    const int f = fl;
    __syncthreads();
    if (!f) {
      found = k;
      break;
    }
    r = r * rho;
  }
  if (tid == 0) kout[blockIdx.x] = found;
}

// Z^{-1} for blocks of order 64 < n <= 128: Z padded with the identity to
// 128 and factored by the tile routine, Z = L L^T with L = [[L11, 0], [L21,
// L22]]; X = L^{-1} = [[X11, 0], [X21, X22]] with X21 = -X22 L21 X11; then
// Z^{-1} = X^T X, whose blocks X11^T X11 + X21^T X21, X22^T X21 and
// X22^T X22 are MFMA products written upper triangle and mirror (exactly
// symmetric).  A non-positive pivot sets F_ZFAIL.
__global__ void __launch_bounds__(256) k_cholinv_tile(const BlkDesc* __restrict__ blks, int* flags,
                                                      const double* __restrict__ Z, double* Zi) {
  __shared__ double sA[kNB * kLD];   // A_11 -> L_11; later X_22
  __shared__ double sX[kNB * kLD];   // X_11
  __shared__ double sB[kNB * kLD];   // A_21 -> L_21 -> L_21 X_11
  __shared__ double sC[kNB * kLD];   // A_22 -> S -> L_22 -> X_21
  __shared__ int fl;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kNB || bd.n > 2 * kNB) return;   // k_cholinv16 / k_cholinv
  if (!(flags[bd.sys] & F_ACTIVE)) return;
  const int n = bd.n, tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  const double* Zb = Z + bd.off;
  auto zpad = [&](int i, int j) { return i < n && j < n ? Zb[i * n + j] : (i == j ? 1.0 : 0.0); };
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int i = e >> 6, j = e & 63;
    sA[i * kLD + j] = zpad(i, j);
    sX[i * kLD + j] = 0.0;
    sB[i * kLD + j] = zpad(kNB + i, j);
    sC[i * kLD + j] = zpad(kNB + i, kNB + j);
  }
  if (tid == 0) fl = 0;
  __syncthreads();
  // products of 64 x 64 tiles in LDS (wave w: rows 16w..16w+15): XYt = X Y^T,
  // XY = X Y, XtY = X^T Y
  auto XYt = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * kLD + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Y[(16 * u + r16) * kLD + k0 + kq], acc[u], 0, 0, 0);
    }
  };
  auto XY = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * kLD + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Y[(k0 + kq) * kLD + 16 * u + r16], acc[u], 0, 0, 0);
    }
  };
  auto XtY = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(k0 + kq) * kLD + 16 * w + r16];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Y[(k0 + kq) * kLD + 16 * u + r16], acc[u], 0, 0, 0);
    }
  };
  // result register q of lane l, tile u: row 16w + 4q + kq, column 16u + r16
  auto put = [&](double* D, const v4d* acc, double sg) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) D[(16 * w + 4 * q + kq) * kLD + 16 * u + r16] = sg * acc[u][q];
  };
  diag_tile(sA, sX, &fl);   // L_11, X_11
  __syncthreads();
  {
    v4d acc[4] = {};
    XYt(sB, sX, acc);       // L_21 = A_21 X_11^T
    __syncthreads();
    put(sB, acc, 1.0);
    __syncthreads();
    v4d upd[4] = {};
    XYt(sB, sB, upd);       // L_21 L_21^T
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) sC[(16 * w + 4 * q + kq) * kLD + 16 * u + r16] -= upd[u][q];
  }
  for (int e = tid; e < kNB * kNB; e += 256) sA[(e >> 6) * kLD + (e & 63)] = 0.0;
  __syncthreads();
  diag_tile(sC, sA, &fl);   // L_22 (sC), X_22 (sA)
  __syncthreads();
  if (tid == 0 && fl) atomicOr(&flags[bd.sys], F_ZFAIL);
  {
    v4d acc[4] = {};
    XY(sB, sX, acc);        // T = L_21 X_11
    __syncthreads();
    put(sB, acc, 1.0);
    __syncthreads();
    v4d x21[4] = {};
    XY(sA, sB, x21);        // X_21 = -X_22 T
    __syncthreads();
    put(sC, x21, -1.0);
    __syncthreads();
  }
  double* out = Zi + bd.off;
  auto store_sym = [&](const v4d* acc, int r0, int c0, bool diag) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + 16 * w + 4 * q + kq, c = c0 + 16 * u + r16;
        if (r >= n || c >= n || (diag && c < r)) continue;
        out[r * n + c] = acc[u][q];
        out[c * n + r] = acc[u][q];
      }
  };
  {
    v4d z11[4] = {};
    XtY(sX, sX, z11);       // X_11^T X_11 + X_21^T X_21
    XtY(sC, sC, z11);
    store_sym(z11, 0, 0, true);
    v4d z21[4] = {};
    XtY(sA, sC, z21);       // X_22^T X_21 (rows 64.., columns ..64)
    store_sym(z21, kNB, 0, false);
    v4d z22[4] = {};
    XtY(sA, sA, z22);       // X_22^T X_22
    store_sym(z22, kNB, kNB, true);
  }
}

void launch_cholinv_tile(hipStream_t st, int nblk, const BlkDesc* blks, int* flags, const double* Z,
                         double* Zi) {
  hipLaunchKernelGGL(k_cholinv_tile, dim3(nblk), dim3(256), 0, st, blks, flags, Z, Zi);
}

// Certificate for blocks of order 64 < n <= 128: pass = Q_j = B^T(y)_j
// passes Cholesky; margin_j = lambda_min(Q_j) / s_j by bisection on the
// Cholesky of Q_j - tau s_j I, each test the tile routine on Q_j padded with
// the identity to 128 (the steps of the column-test kernel otherwise).
__global__ void __launch_bounds__(256) k_certificate_tile(const BlkDesc* __restrict__ blks,
                                                          const SysDesc* __restrict__ sys,
                                                          const int* __restrict__ flags,
                                                          const double* __restrict__ Q, int iters,
                                                          double* out) {
  __shared__ double sA[kNB * kLD];
  __shared__ double sX[kNB * kLD];
  __shared__ double sB[kNB * kLD];
  __shared__ double sC[kNB * kLD];
  __shared__ int fl;
  __shared__ double fro;
  const BlkDesc bd = blks[blockIdx.x];
  if (bd.n <= kNB || bd.n > 2 * kNB) return;   // k_certificate16 / k_certificate
  if (!(flags[bd.sys] & F_ACTIVE)) return;
  const SysDesc sd = sys[bd.sys];
  const int n = bd.n, nn = n * n, tid = threadIdx.x;
  const double sj = sd.scale[bd.j];
  const double* Qb = Q + bd.off;
  if (tid == 0) {
    double f = 0;
    for (int e = 0; e < nn; ++e) f += Qb[e] * Qb[e];
    fro = sqrt(f);
  }
  auto entry = [&](int i, int j, double shift) {
    if (i < n && j < n) return i == j ? Qb[i * n + j] - shift : Qb[i * n + j];
    return i == j ? 1.0 : 0.0;
  };
  double lo = 0, hi = 0;
  int pass0 = 0;
  for (int it = -1; it < iters; ++it) {
    const double tau = it < 0 ? 0.0 : 0.5 * (lo + hi);
    __syncthreads();
    const double shift = tau * sj;
    for (int e = tid; e < kNB * kNB; e += 256) {
      const int i = e >> 6, j = e & 63;
      sA[i * kLD + j] = entry(i, j, shift);
      sB[i * kLD + j] = entry(kNB + i, j, shift);
      sC[i * kLD + j] = entry(kNB + i, kNB + j, shift);
    }
    if (tid == 0) fl = 0;
    tile_chol_test(sA, sX, sB, sC, &fl);
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
  if (tid == 0) {
    out[blockIdx.x * 2 + 0] = pass0;
    out[blockIdx.x * 2 + 1] = 0.5 * (lo + hi);
  }
}

void launch_certificate_tile(hipStream_t st, int nblk, const BlkDesc* blks, const SysDesc* sys,
                             const int* flags, const double* Q, int iters, double* out) {
  hipLaunchKernelGGL(k_certificate_tile, dim3(nblk), dim3(256), 0, st, blks, sys, flags, Q, iters, out);
}

void launch_ladder_tile(hipStream_t st, int nblk, const BlkDesc* blks, const int* flags, const double* V,
                        const double* dV, double rho, double frac, int len, int* kout) {
  hipLaunchKernelGGL(k_ladder_tile, dim3(nblk), dim3(256), 0, st, blks, flags, V, dV, rho, frac, len, kout);
}

// Diagonal step p: one workgroup per system factors the 64 x 64 tile A_pp
// and inverts the factor, storing L_pp and L_pp^{-1}.  (Inside a
// super-panel the narrow update of step p - 1 does this instead.)
__global__ void __launch_bounds__(256) k_chol_diag(const SysDesc* __restrict__ sys, int* flags,
                                                   const double* __restrict__ Lam, double* Ldiag,
                                                   double* Linv, const int* __restrict__ st_sys,
                                                   int p) {
  __shared__ double sA[kNB * kLD];
  __shared__ double sX[kNB * kLD];
  __shared__ int fl;
  const int s = st_sys[blockIdx.x];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  const double* App = Lam + sd.loff + (int64_t)p * kNB * ld + (int64_t)p * kNB;
  const int tid = threadIdx.x;
  if (tid == 0) fl = 0;
  double ld16[kNB * kNB / 256];   // all loads in flight before the LDS stores
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    ld16[it] = App[(int64_t)(e >> 6) * ld + (e & 63)];
  }
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    const int r = e >> 6, cc = e & 63;
    sA[r * kLD + cc] = ld16[it];
    sX[r * kLD + cc] = 0.0;
  }
  __syncthreads();
  diag_tile(sA, sX, &fl);
  store_diag(sA, sX, Ldiag + sd.dgoff + (int64_t)p * kNB * kNB, Linv + sd.dgoff + (int64_t)p * kNB * kNB);
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
  double la[kNB * kNB / 256], lx[kNB * kNB / 256];   // all loads in flight first
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    la[it] = Ai[(int64_t)(e >> 6) * ld + (e & 63)];
    lx[it] = Xg[e];
  }
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    const int r = e >> 6, c = e & 63;
    sA[r * LDT + c] = la[it];
    sX[r * LDT + c] = lx[it];
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
// The workgroup of tile (p+1, p+1) then factors and inverts it (the diagonal
// step of p + 1), overlapped with the other tiles' updates.
__global__ void __launch_bounds__(256, 2) k_chol_update(const SysDesc* __restrict__ sys,
                                                     int* flags, double* Lam, double* Ldiag,
                                                     double* Linv, const int* __restrict__ st_sys,
                                                     const int* __restrict__ st_pre, int cnt,
                                                     int p) {
  __shared__ double sa[kNB * LDT];
  __shared__ double sb[kNB * LDT];
  __shared__ int fl;
  // the first cnt workgroups take tile (p+1, p+1) of each system, so that the
  // diagonal steps start first; the rest follow system by system
  int si, t;
  if ((int)blockIdx.x < cnt) {
    si = blockIdx.x;
    t = 0;
  } else {
    const int b = blockIdx.x - cnt;   // last si with st_pre[si] - si <= b
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st_pre[mid] - mid <= b) lo = mid;
      else hi = mid - 1;
    }
    si = lo;
    t = 1 + b - (st_pre[si] - si);
  }
  const int s = st_sys[si];
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
  double la[kNB * kNB / 256], lb[kNB * kNB / 256];   // all loads in flight first
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    la[it] = Li[(int64_t)(e >> 6) * ld + (e & 63)];
    lb[it] = Lj[(int64_t)(e >> 6) * ld + (e & 63)];
  }
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    const int r = e >> 6, c = e & 63;
    sa[r * LDT + c] = la[it];
    sb[r * LDT + c] = lb[it];
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
  double cv[16];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[u * 4 + q] = C[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cc = 16 * u + r16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = 16 * w + 4 * q + kq;
      if (i != j || cc <= rr) C[(int64_t)rr * ld + cc] = cv[u * 4 + q] - acc[u][q];
    }
  }
  if (t != 0) return;   // tile (p+1, p+1): the next diagonal step
  if (tid == 0) fl = 0;
  __syncthreads();      // the operand panels are no longer read
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sa[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = cv[u * 4 + q] - acc[u][q];
#pragma unroll
  for (int it = 0; it < kNB * kNB / 256; ++it) {
    const int e = tid + 256 * it;
    sb[(e >> 6) * LDT + (e & 63)] = 0.0;
  }
  __syncthreads();
  diag_tile(sa, sb, &fl);
  store_diag(sa, sb, Ldiag + sd.dgoff + (int64_t)j * kNB * kNB, Linv + sd.dgoff + (int64_t)j * kNB * kNB);
  if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
}

// Look-ahead right-looking step p (systems factored as one super-panel).  On
// entry column p holds L and L_pp^{-1} is stored.  Light workgroups update
// the tiles right of column p + 1, A_ij -= L_ip L_jp^T (j >= p + 2).  Heavy
// workgroups, one per tile (i, p+1) with i >= p + 1 and dispatched first,
// each form the updated diagonal tile A_{p+1,p+1} - L_{p+1,p} L_{p+1,p}^T
// and factor and invert it: the same operations on the same operands in
// every such workgroup, so the same bits.  The diagonal tile's workgroup
// stores L_{p+1,p+1} and its inverse; the others apply the inverse to their
// own updated tile, L_{i,p+1} = (A_{i,p+1} - L_ip L_{p+1,p}^T) L_{p+1,p+1}^{-T}.
// On return column p + 1 is factored: one launch per step, the next
// column's panel solve done beside the update rather than after it, for the
// price of the diagonal factorisation repeated by the column's workgroups.
// Every value is computed as the right-looking steps compute it; the matrix's
// diagonal tiles keep their values from before the last update (the factor
// is read from Ldiag).
__global__ void __launch_bounds__(256, 2) k_chol_look(const SysDesc* __restrict__ sys, int* flags, double* Lam,
                                                   double* Ldiag, double* Linv,
                                                   const int* __restrict__ h_sys, const int* __restrict__ h_pre,
                                                   int hcnt, int htot, const int* __restrict__ l_sys,
                                                   const int* __restrict__ l_pre, int lcnt, int p) {
  __shared__ double sa[kNB * LDT];
  __shared__ double sb[kNB * LDT];
  __shared__ int fl;
  constexpr int NE = kNB * kNB / 256;
  const bool heavy = (int)blockIdx.x < htot;
  const int b = heavy ? (int)blockIdx.x : (int)blockIdx.x - htot;
  const int si = heavy ? find_owner(h_pre, hcnt, b) : find_owner(l_pre, lcnt, b);
  const int s = heavy ? h_sys[si] : l_sys[si];
  const int t = b - (heavy ? h_pre[si] : l_pre[si]);
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  int i, j;
  if (heavy) {
    j = p + 1;
    i = j + t;
  } else {
    // column j = p + 2 + c, rows i = j .. P-1: column c holds R - c tiles,
    // R = P - p - 2
    const int R = sd.P - p - 2;
    int c = 0, base = 0;
    while (t >= base + (R - c)) { base += R - c; ++c; }
    j = p + 2 + c;
    i = j + (t - base);
  }
  auto tile = [&](int r, int cc) { return A + (int64_t)r * kNB * ld + (int64_t)cc * kNB; };
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  {
    const double* Li = tile(i, p);
    const double* Lj = tile(j, p);
    double la[NE], lb[NE];   // all loads in flight first
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      la[it] = Li[(int64_t)(e >> 6) * ld + (e & 63)];
      lb[it] = Lj[(int64_t)(e >> 6) * ld + (e & 63)];
    }
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      sa[(e >> 6) * LDT + (e & 63)] = la[it];
      sb[(e >> 6) * LDT + (e & 63)] = lb[it];
    }
  }
  __syncthreads();
  // acc = X Y^T for 64 x 64 tiles X, Y in LDS (wave w: rows 16w..16w+15)
  auto prodT = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double bv = Y[(16 * u + r16) * LDT + k0 + kq];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[u], 0, 0, 0);
      }
    }
  };
  auto ld_tile = [&](double* v, const double* T) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[u * 4 + q] = T[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16];
  };
  double* C = tile(i, j);
  v4d acc[4] = {};
  double cv[16];
  if (!heavy) {
    prodT(sa, sb, acc);
    ld_tile(cv, C);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = 16 * u + r16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 16 * w + 4 * q + kq;
        if (i != j || cc <= rr) C[(int64_t)rr * ld + cc] = cv[u * 4 + q] - acc[u][q];
      }
    }
    return;
  }
  // heavy: E = A_{i,p+1} - L_ip L_{p+1,p}^T (below the diagonal) and the
  // updated diagonal tile D = A_{p+1,p+1} - L_{p+1,p} L_{p+1,p}^T
  double ev[16];
  if (i != j) {
    prodT(sa, sb, acc);
    ld_tile(cv, C);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) ev[u * 4 + q] = cv[u * 4 + q] - acc[u][q];
  }
  v4d dacc[4] = {};
  prodT(sb, sb, dacc);
  double dv[16];
  ld_tile(dv, tile(j, j));
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) dv[u * 4 + q] -= dacc[u][q];
  // (D is not written back: the column's other workgroups read the tile's
  // values before this step's update; factor and inverse go to Ldiag / Linv)
  if (tid == 0) fl = 0;
  __syncthreads();   // the operand panels are no longer read
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sa[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = dv[u * 4 + q];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    sb[(e >> 6) * LDT + (e & 63)] = 0.0;
  }
  __syncthreads();
  diag_tile(sa, sb, &fl);   // sa: L_{p+1,p+1}, sb: its inverse
  if (i == j) {
    store_diag(sa, sb, Ldiag + sd.dgoff + (int64_t)j * kNB * kNB, Linv + sd.dgoff + (int64_t)j * kNB * kNB);
    if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
    return;
  }
  __syncthreads();   // sa (the factor) is not needed here: E goes there
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sa[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = ev[u * 4 + q];
  __syncthreads();
  v4d lacc[4] = {};
  prodT(sa, sb, lacc);   // L_{i,p+1}[r][c] = sum_k E[r][k] X[c][k]
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) C[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16] = lacc[u][q];
}

// Right-looking step p with the panel solve folded in (systems factored as
// one super-panel): every workgroup of tile (i, j), j > p, forms the panel
// tiles it needs, L_ip = C_ip L_pp^{-T} and L_jp, from the column the
// previous step left and L_pp^{-1}, then C_ij -= L_ip L_jp^T; the workgroup
// of tile (p+1, p+1) (dispatched first) goes on to factor it.  So a step is
// one launch instead of a triangular solve and an update.  Column p is read
// by many workgroups of the step, so its L tiles go to a two-slot panel
// buffer (slot p % 2, written by the workgroups of column p + 1) and reach
// the matrix one step later (copied by the workgroups of column p + 2 and
// the diagonal one); the last step writes its single tile directly.
__global__ void __launch_bounds__(256, 2) k_chol_fused(const SysDesc* __restrict__ sys, int* flags, double* Lam,
                                                    double* Ldiag, double* Linv, double* PB,
                                                    const int* __restrict__ st_sys,
                                                    const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sX[kNB * LDT];
  __shared__ double sA[kNB * LDT];
  __shared__ int fl;
  constexpr int NE = kNB * kNB / 256;
  int si, t;
  if ((int)blockIdx.x < cnt) {
    si = blockIdx.x;
    t = 0;
  } else {
    const int b = blockIdx.x - cnt;   // last si with st_pre[si] - si <= b
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st_pre[mid] - mid <= b) lo = mid;
      else hi = mid - 1;
    }
    si = lo;
    t = 1 + b - (st_pre[si] - si);
  }
  const int s = st_sys[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  const int P = sd.P, R = P - p - 1;
  int c = 0, base = 0;
  while (t >= base + (R - c)) { base += R - c; ++c; }
  const int j = p + 1 + c, i = j + (t - base);
  const bool own = i == j;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  auto tile = [&](int r, int cc) { return A + (int64_t)r * kNB * ld + (int64_t)cc * kNB; };
  double* pb = PB + sd.pboff;
  auto slot = [&](int q, int r) { return pb + ((int64_t)(q & 1) * P + r) * kNB * kNB; };
  auto gload = [&](double* v, const double* src, int64_t lds) {
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      v[it] = src[(int64_t)(e >> 6) * lds + (e & 63)];
    }
  };
  auto sstore = [&](double* dst, const double* v) {
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      dst[(e >> 6) * LDT + (e & 63)] = v[it];
    }
  };
  auto prodT = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double b = Y[(16 * u + r16) * LDT + k0 + kq];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  };
  auto to_lds = [&](double* dst, const v4d* acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = acc[u][q];
  };
  auto to_tile = [&](double* dst, int64_t lds, const v4d* acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(int64_t)(16 * w + 4 * q + kq) * lds + 16 * u + r16] = acc[u][q];
  };
  auto copy_tile = [&](double* dst, const double* src) {   // panel slot -> matrix
    double v[NE];
    gload(v, src, kNB);
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      dst[(int64_t)(e >> 6) * ld + (e & 63)] = v[it];
    }
  };
  // operands in registers first: L_pp^{-1}, C_ip, C_jp (C_ij later, in
  // flight during the last product)
  double vx[NE], va[NE], vb[NE], cv[NE];
  gload(vx, Linv + sd.dgoff + (int64_t)p * kNB * kNB, kNB);
  gload(va, tile(i, p), ld);
  if (!own) gload(vb, tile(j, p), ld);
  double* C = tile(i, j);
  // the previous step's panel tiles of this row (and, for the diagonal
  // workgroup, of row p) into the matrix
  if (p >= 1 && j == p + 1) {
    copy_tile(tile(i, p - 1), slot(p - 1, i));
    if (own) copy_tile(tile(p, p - 1), slot(p - 1, p));
  }
  sstore(sX, vx);
  sstore(sA, va);
  __syncthreads();
  v4d li[4] = {}, lj[4] = {};
  prodT(sA, sX, li);
  if (!own) {
    __syncthreads();
    sstore(sA, vb);
    __syncthreads();
    prodT(sA, sX, lj);
  }
  if (j == p + 1) {
    if (p == P - 2) to_tile(tile(i, p), ld, li);   // the last step's only tile
    else to_tile(slot(p, i), kNB, li);
  }
  __syncthreads();
  to_lds(sA, li);
  if (!own) to_lds(sX, lj);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[u * 4 + q] = C[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16];
  __syncthreads();
  v4d acc[4] = {};
  prodT(sA, own ? sA : sX, acc);
  if (t != 0) {   // every tile but (p+1, p+1); diagonal ones keep their upper part
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = 16 * u + r16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 16 * w + 4 * q + kq;
        if (!own || cc <= rr) C[(int64_t)rr * ld + cc] = cv[u * 4 + q] - acc[u][q];
      }
    }
    return;
  }
  // tile (p+1, p+1): the next diagonal step
  if (tid == 0) fl = 0;
  __syncthreads();   // the product's operands are no longer read
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sA[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = cv[u * 4 + q] - acc[u][q];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    sX[(e >> 6) * LDT + (e & 63)] = 0.0;
  }
  __syncthreads();
  diag_tile(sA, sX, &fl);
  store_diag(sA, sX, Ldiag + sd.dgoff + (int64_t)j * kNB * kNB, Linv + sd.dgoff + (int64_t)j * kNB * kNB);
  if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
}

// Wide update at the end of a super-panel of sw panels (p = its last
// panel): A_ij -= sum over the super-panel's panels q of L_iq L_jq^T for every
// tile pair right of it (depth 64 sw), on 128 x 128 output blocks (2 x 2
// tiles; wave w owns the 64 x 64 quadrant (w/2, w%2) as 4 x 4 MFMA tiles).
// The depth is staged through two LDS buffers 16 columns at a time, the
// chunk after next prefetched into registers; 70 KB of LDS and at most 256
// registers per lane let two workgroups share a compute unit.  Only the
// lower triangle (column <= row) of the matrix is written; rows or columns
// past Kpad are skipped.
//
// Block order: the dispatcher hands consecutive workgroups to the eight
// XCDs in turn, so workgroup b is renumbered to give each XCD one
// contiguous range of the block list; the list walks groups of kWG block
// rows column by column, so that an XCD's L2 keeps the group's row panels
// while each column panel is read once per group.
constexpr int kWT = 128, kWK = 16, kWLD = kWK + 1;
constexpr int kWRP = 256 / kWK;          // rows staged per pass
constexpr int kWU = kWT / kWRP;          // passes (values per thread and operand)
constexpr int kWG = 4;                   // block rows per group of the block order

// (bi, bj), bj <= bi < nb, of position t of the grouped block order
__device__ inline void wide_block(int t, int nb, int& bi, int& bj) {
  // group k holds rows k kWG .. k kWG + kWG - 1; kWG k (kWG k + 1) / 2 blocks precede it
  int k = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5) / kWG;
  while (k > 0 && (kWG * k) * (kWG * k + 1) / 2 > t) --k;
  while ((kWG * (k + 1)) * (kWG * (k + 1) + 1) / 2 <= t) ++k;
  const int r0 = kWG * k, r1 = min(r0 + kWG, nb) - 1, h = r1 - r0 + 1;
  int u = t - r0 * (r0 + 1) / 2;
  if (u < (r0 + 1) * h) {   // columns 0 .. r0: every row of the group
    bj = u / h;
    bi = r0 + u % h;
    return;
  }
  u -= (r0 + 1) * h;        // column r0 + j holds the rows r0 + j .. r1
  int j = 1;
  while (u >= h - j) {
    u -= h - j;
    ++j;
  }
  bj = r0 + j;
  bi = bj + u;
}

// (bi, bj) of position t among the blocks bj < ncb, bj <= bi < nrb: groups of
// kWG block rows, column by column inside a group (the blocks of a sub-panel
// update: every row below it, the columns up to the end of its super-panel)
__device__ inline void tall_block(int t, int nrb, int ncb, int& bi, int& bj) {
  int r0 = 0;
  // groups that reach the diagonal of the column range
  while (r0 < ncb && r0 < nrb) {
    const int r1 = min(r0 + kWG, nrb) - 1, cend = min(ncb, r1 + 1);
    int cnt = 0;
    for (int c = 0; c < cend; ++c) cnt += r1 - max(r0, c) + 1;
    if (t < cnt) {
      for (int c = 0; c < cend; ++c) {
        const int h = r1 - max(r0, c) + 1;
        if (t < h) {
          bj = c;
          bi = max(r0, c) + t;
          return;
        }
        t -= h;
      }
    }
    t -= cnt;
    r0 += kWG;
  }
  // below them every group is a full h x ncb rectangle
  const int g = t / (kWG * ncb);
  r0 += kWG * g;
  t -= g * kWG * ncb;
  const int h = min(r0 + kWG, nrb) - r0;
  bj = t / h;
  bi = r0 + t % h;
}

// last panel of the super-panel of panel q (a super-panel followed by fewer
// than sw panels absorbs them); the host tables use the same rule
__device__ inline int sp_end_dev(int P, int q, int sw) {
  const int se = (q / sw) * sw + sw - 1;
  return P - 1 - se < sw ? P - 1 : se;
}

// mode 0: the update after super-panel p (depth sw panels, every tile right
// of it); mode 1: the update after sub-panel p inside a super-panel (depth
// ssw panels, the rows below it and only the columns up to the end of the
// super-panel, whose own update adds the whole super-panel later).  The
// look-ahead splits mode 0 in two: mode 2, the next super-panel's columns
// (every row below p), and mode 3, every tile right of the next super-panel
// (run beside that super-panel's steps).
__global__ void __launch_bounds__(256, 2) k_chol_update_wide(const SysDesc* __restrict__ sys,
                                                             const int* __restrict__ flags, double* Lam,
                                                             const int* __restrict__ st_sys,
                                                             const int* __restrict__ st_pre, int cnt,
                                                             int p, int mode) {
  __shared__ double sa[2][kWT * kWLD];   // two stages: one is multiplied while
  __shared__ double sb[2][kWT * kWLD];   // the next is written
  const int g = xcd_order(blockIdx.x, gridDim.x);
  const int si = find_owner(st_pre, cnt, g);
  const int s = st_sys[si];
  const int t = g - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  int bi, bj, cmax = sd.Kpad, dpan = sd.sw, q0 = p + 1;
  const int nrb = (sd.P - p - 1 + 1) / 2;
  if (mode == 1 || mode == 2) {
    // the tall block range: every row below p, the columns up to the end of
    // the super-panel of p (mode 1) or of the next one (mode 2)
    const int se = sp_end_dev(sd.P, mode == 1 ? p : p + 1, sd.sw);
    tall_block(t, nrb, (se - p + 1) / 2, bi, bj);
    cmax = kNB * (se + 1);
    if (mode == 1) dpan = sd.ssw;
  } else if (mode == 3) {
    const int ne = sp_end_dev(sd.P, p + 1, sd.sw);
    q0 = ne + 1;
    wide_block(t, (sd.P - ne) / 2, bi, bj);
  } else {
    wide_block(t, nrb, bi, bj);
  }
  const int r0 = kNB * (q0 + 2 * bi), c0 = kNB * (q0 + 2 * bj);
  const int nmax = sd.Kpad;
  const int d0 = kNB * (p - dpan + 1), D = kNB * dpan;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // staging map: thread loads rows tid / kWK + kWRP u, column tid % kWK
  const int lr = tid / kWK, lk = tid % kWK;
  double ra[kWU], rb[kWU];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      // rows past Kpad (second half of an edge block) read the last row
      // instead, so the loads need no branches; what they contribute lands
      // only in rows or columns of the block that are not stored.  Nothing
      // uses the values before they are staged one chunk later, so the
      // loads stay in flight across the chunk's products.
      const int row = lr + kWRP * u;
      const int ra_r = min(r0 + row, nmax - 1), rb_r = min(c0 + row, nmax - 1);
      ra[u] = A[(int64_t)ra_r * ld + d0 + kc + lk];
      rb[u] = A[(int64_t)rb_r * ld + d0 + kc + lk];
    }
  };
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      sa[buf][(lr + kWRP * u) * kWLD + lk] = ra[u];
      sb[buf][(lr + kWRP * u) * kWLD + lk] = rb[u];
    }
  };
  // chunk kc is multiplied from buffer cur while chunk kc + kWK (loaded one
  // chunk earlier) is written to the other buffer and chunk kc + 2 kWK is
  // loaded; one barrier per chunk
  load(0);
  stage(0);
  if (kWK < D) load(kWK);
  __syncthreads();
  for (int kc = 0, cur = 0; kc < D; kc += kWK, cur ^= 1) {
#pragma unroll
    for (int ks = 0; ks < kWK; ks += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sa[cur][(wr + 16 * a + r16) * kWLD + ks + kq];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sb[cur][(wc + 16 * b + r16) * kWLD + ks + kq];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (kc + kWK < D) {
      stage(cur ^ 1);
      if (kc + 2 * kWK < D) load(kc + 2 * kWK);
    }
    __syncthreads();
  }
  // C -= acc, one 16-row stripe at a time: all sixteen loads of a stripe are
  // issued before any store (clamped addresses; masked stores)
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double cv[16];
    int64_t ix[16];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int R = r0 + wr + 16 * a + 4 * q + kq;
        const int Cc = c0 + wc + 16 * b + r16;
        ix[b * 4 + q] = (int64_t)min(R, nmax - 1) * ld + min(Cc, nmax - 1);
        cv[b * 4 + q] = A[ix[b * 4 + q]];
      }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int R = r0 + wr + 16 * a + 4 * q + kq;
        const int Cc = c0 + wc + 16 * b + r16;
        if (R < nmax && Cc < cmax && Cc <= R) A[ix[b * 4 + q]] = cv[b * 4 + q] - acc[a][b][q];
      }
  }
}

// Left-looking factorisation for systems with few tiles: one launch per tile
// column j, one workgroup per tile (i, j), i >= j, of every system in it.
// The workgroup first forms the previous column's factor tiles it needs,
// L_{i,j-1} = C_{i,j-1} L_{j-1,j-1}^{-T} and L_{j,j-1} (column j-1 holds the
// updated tiles C the previous launch left), then
//   C_ij = A_ij - sum_{k < j} L_ik L_jk^T
// (the k = j-1 term from those two tiles, the rest read from the stored
// factor), and the diagonal workgroup factors and inverts C_jj.  Each tile is
// thus updated once, with one pass of depth 64 j, and a factorisation takes P
// launches instead of a triangular solve and an update per tile column.
// Stores: L_{i,j-1} for i > j (nobody else in the launch reads row i); row
// j's tile L_{j,j-1} is read as C by every workgroup of the launch, so the
// next launch stores it (its last workgroup, off the diagonal workgroup's
// longer path), or this one's diagonal workgroup when j is the last column.
// The tiles of the next k are loaded into registers while the current
// product runs.
__global__ void __launch_bounds__(256) k_chol_left(const SysDesc* __restrict__ sys, int* flags, double* Lam,
                                                   double* Ldiag, double* Linv,
                                                   const int* __restrict__ st_sys,
                                                   const int* __restrict__ st_pre, int cnt, int j) {
  __shared__ double sX[kNB * LDT];
  __shared__ double sA[kNB * LDT];
  __shared__ double sB[kNB * LDT];
  __shared__ int fl;
  constexpr int NE = kNB * kNB / 256;   // tile elements per thread
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  const double* Li = Linv + sd.dgoff;
  const int P = sd.P, i = j + t;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  auto tile = [&](int r, int c) { return A + (int64_t)r * kNB * ld + (int64_t)c * kNB; };
  auto gload = [&](double* v, const double* src, int64_t lds) {
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      v[it] = src[(int64_t)(e >> 6) * lds + (e & 63)];
    }
  };
  auto sstore = [&](double* dst, const double* v) {
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      dst[(e >> 6) * LDT + (e & 63)] = v[it];
    }
  };
  // acc += X Y^T for the wave's 16 rows of X (FP64 MFMA)
  auto prodT = [&](const double* X, const double* Y, v4d* acc) {
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = X[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double b = Y[(16 * u + r16) * LDT + k0 + kq];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  };
  auto to_lds = [&](double* dst, const v4d* acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = acc[u][q];
  };
  auto to_global = [&](double* dst, const v4d* acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16] = acc[u][q];
  };
  const bool own = i == j;   // the diagonal workgroup: row i is row j
  double* C = tile(i, j);
  double cv[NE];             // C_ij in the accumulator layout
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[u * 4 + q] = C[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16];
  // L_{j-1,j-2}, which the previous launch's workgroups formed for themselves
  if (j >= 2 && i == (j < P - 1 ? P - 1 : j)) {
    double vx[NE], vc[NE];
    gload(vx, Li + (int64_t)(j - 2) * kNB * kNB, kNB);
    gload(vc, tile(j - 1, j - 2), ld);
    sstore(sX, vx);
    sstore(sA, vc);
    __syncthreads();
    v4d l[4] = {};
    prodT(sA, sX, l);
    to_global(tile(j - 1, j - 2), l);
    __syncthreads();
  }
  v4d acc[4] = {};
  if (j >= 1) {
    double va[NE], vb[NE];   // the next k's tiles, in flight during a product
    {
      double vx[NE];
      gload(vx, Li + (int64_t)(j - 1) * kNB * kNB, kNB);
      gload(va, tile(i, j - 1), ld);
      if (!own) gload(vb, tile(j, j - 1), ld);
      sstore(sX, vx);
      sstore(sA, va);
      if (!own) sstore(sB, vb);
    }
    if (j >= 2) {
      gload(va, tile(i, 0), ld);
      if (!own) gload(vb, tile(j, 0), ld);
    }
    __syncthreads();
    v4d li[4] = {}, lj[4] = {};
    prodT(sA, sX, li);
    if (!own) prodT(sB, sX, lj);
    __syncthreads();
    to_lds(sA, li);
    if (!own) to_lds(sB, lj);
    if (i > j || j == P - 1) to_global(tile(i, j - 1), li);
    __syncthreads();
    prodT(sA, own ? sA : sB, acc);
    for (int k = 0; k < j - 1; ++k) {
      __syncthreads();
      sstore(sA, va);
      if (!own) sstore(sB, vb);
      if (k + 1 < j - 1) {
        gload(va, tile(i, k + 1), ld);
        if (!own) gload(vb, tile(j, k + 1), ld);
      }
      __syncthreads();
      prodT(sA, own ? sA : sB, acc);
    }
  }
  if (!own) {
    if (j == 0) return;   // the first column is already C
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        C[(int64_t)(16 * w + 4 * q + kq) * ld + 16 * u + r16] = cv[u * 4 + q] - acc[u][q];
    return;
  }
  // the diagonal tile: C_jj - acc, factored and inverted
  if (tid == 0) fl = 0;
  __syncthreads();   // the product's operands are no longer read
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) sA[(16 * w + 4 * q + kq) * LDT + 16 * u + r16] = cv[u * 4 + q] - acc[u][q];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    sX[(e >> 6) * LDT + (e & 63)] = 0.0;
  }
  __syncthreads();
  diag_tile(sA, sX, &fl);
  store_diag(sA, sX, Ldiag + sd.dgoff + (int64_t)j * kNB * kNB, Linv + sd.dgoff + (int64_t)j * kNB * kNB);
  if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
}

// Whole solve L L^T x = rhs for systems with few tiles: one workgroup of 8
// waves per system sweeps all tile steps (no inter-workgroup dependency); the
// right-hand side and the iterate stay in LDS.  Each pass over a column panel
// of L (the rows below its diagonal tile) gives every group of 16 lanes one
// row at a time, each lane 4 consecutive entries: the forward sweep forms row
// dots (r_i -= L_ip z_p, right-looking), the backward sweep column sums
// (x_p = L_pp^{-T} (z_p - sum_i L_ip^T x_i), left-looking), so both read L
// row-contiguously.  kSvR rows per group are loaded before any is used.
constexpr int kSvT = 512;         // threads
constexpr int kSvG = kSvT / 16;   // lane groups
constexpr int kSvR = 8;           // rows in flight per group

__device__ inline double gsum16(double v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

__device__ inline void ld4(const double* p, double* v) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

// Forward (L z = r) and/or backward (L^T x = z) sweep over the panels p0..p1
// of one system, restricted to the rows and columns of those panels: sr (LDS)
// holds entries p0*64 .. (p1+1)*64 - 1 of the vector and is overwritten by the
// result.  A is the system's matrix (leading dimension ld), Di its stored
// diagonal-tile inverses.  The next panel's L_pp^{-1} rows and first
// kSvG kSvR rows of L below it are loaded before the barrier that ends the
// current panel.
template <bool FWD, bool BWD>
__device__ __forceinline__ void solve_range(const double* __restrict__ A, int64_t ld, const double* __restrict__ Di,
                            int p0, int p1, double* sr, double* sred, double* sv) {
  const int tid = threadIdx.x, g = tid >> 4, j = tid & 15;
  const int base = p0 * kNB, rend = (p1 + 1) * kNB;
  double d0[4], d1[4], a[kSvR][4];
  auto load_di = [&](int q) {
    const double* D = Di + (int64_t)q * kNB * kNB;
    ld4(D + g * kNB + 4 * j, d0);
    ld4(D + (g + kSvG) * kNB + 4 * j, d1);
  };
  auto load_rows = [&](int q, int ib) {
    const double* Lq = A + (int64_t)q * kNB + 4 * j;
#pragma unroll
    for (int m = 0; m < kSvR; ++m) ld4(Lq + (int64_t)min(ib + g + kSvG * m, rend - 1) * ld, a[m]);
  };
  if constexpr (FWD) {
    // z_p = L_pp^{-1} r_p, then r_i -= L_ip z_p below (inside the range)
    load_di(p0);
    if (p0 < p1) load_rows(p0, (p0 + 1) * kNB);
    __syncthreads();
    for (int p = p0; p <= p1; ++p) {
      double rp[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) rp[q] = sr[p * kNB - base + 4 * j + q];
      const double z0 = gsum16(d0[0] * rp[0] + d0[1] * rp[1] + d0[2] * rp[2] + d0[3] * rp[3]);
      const double z1 = gsum16(d1[0] * rp[0] + d1[1] * rp[1] + d1[2] * rp[2] + d1[3] * rp[3]);
      __syncthreads();   // r_p read by every group
      if (j == 0) {
        sr[p * kNB - base + g] = z0;
        sr[p * kNB - base + g + kSvG] = z1;
      }
      __syncthreads();
      double zp[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) zp[q] = sr[p * kNB - base + 4 * j + q];
      for (int ib = (p + 1) * kNB; ib < rend; ib += kSvG * kSvR) {
        if (ib != (p + 1) * kNB) load_rows(p, ib);
#pragma unroll
        for (int m = 0; m < kSvR; ++m) {
          const double t = gsum16(a[m][0] * zp[0] + a[m][1] * zp[1] + a[m][2] * zp[2] + a[m][3] * zp[3]);
          const int i = ib + g + kSvG * m;
          if (j == 0 && i < rend) sr[i - base] -= t;
        }
      }
      if (p < p1) {
        load_di(p + 1);
        if (p + 1 < p1) load_rows(p + 1, (p + 2) * kNB);
      }
      __syncthreads();
    }
  }
  if constexpr (BWD) {
    // x_p = L_pp^{-T} (z_p - sum_{i below, inside the range} L_ip^T x_i)
    load_di(p1);
    __syncthreads();
    for (int p = p1; p >= p0; --p) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int ib = (p + 1) * kNB; ib < rend; ib += kSvG * kSvR) {
        if (ib != (p + 1) * kNB) load_rows(p, ib);
        double xv[kSvR];
#pragma unroll
        for (int m = 0; m < kSvR; ++m) {
          const int i = ib + g + kSvG * m;
          xv[m] = i < rend ? sr[i - base] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < kSvR; ++m)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += a[m][q] * xv[m];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) sred[g * kNB + 4 * j + q] = acc[q];
      __syncthreads();
      if (tid < kNB) {
        double t = sr[p * kNB - base + tid];
        for (int gg = 0; gg < kSvG; ++gg) t -= sred[gg * kNB + tid];
        sv[tid] = t;
      }
      __syncthreads();
      const double v0 = sv[g], v1 = sv[g + kSvG];
#pragma unroll
      for (int q = 0; q < 4; ++q) sred[g * kNB + 4 * j + q] = d0[q] * v0 + d1[q] * v1;
      if (p > p0) {
        load_di(p - 1);
        load_rows(p - 1, p * kNB);
      }
      __syncthreads();
      if (tid < kNB) {
        double t = 0.0;
        for (int gg = 0; gg < kSvG; ++gg) t += sred[gg * kNB + tid];
        sr[p * kNB - base + tid] = t;
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kSvT) k_trsv_small(const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const int* __restrict__ small_ids,
                                                     const double* __restrict__ Lam,
                                                     const double* __restrict__ Linv,
                                                     const double* __restrict__ rhs, double* x) {
  __shared__ double sr[kNB * kSmallP];   // r, overwritten by z, then by x
  __shared__ double sred[kSvG * kNB];    // per-group partial column sums
  __shared__ double sv[kNB];
  const int s = small_ids[blockIdx.x];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  for (int k = threadIdx.x; k < sd.Kpad; k += kSvT) sr[k] = rhs[sd.voff + k];
  solve_range<true, false>(Lam + sd.loff, sd.Kpad, Linv + sd.dgoff, 0, sd.P - 1, sr, sred, sv);
  solve_range<false, true>(Lam + sd.loff, sd.Kpad, Linv + sd.dgoff, 0, sd.P - 1, sr, sred, sv);
  for (int k = threadIdx.x; k < sd.Kpad; k += kSvT) x[sd.voff + k] = sr[k];
}

// Larger systems solve by groups of kSG panels (kGS rows).  After the
// factorisation, k_trsv_ginv forms the inverse of each group's diagonal block
// of the factor, G_q = L_qq^{-1}, and its transpose.  Forward, group q:
// z_q = G_q r_q (k_trsv_gapply, many workgroups), then r_i -= L_{i,q} z_q for
// every row tile below the group (k_trsv_gfwd).  Backward, groups in reverse:
// x_q = G_q^T z_q, then z_c -= L_{q,c}^T x_q for every column tile left of it
// (k_trsv_gbwd).  Every launch reads its part of L at full width; the only
// serial chain is the one between groups.
//
// G_q by recursive doubling over its 64 x 64 tiles, starting from the stored
// inverses L_ii^{-1} of the diagonal tiles.  For a block split in halves A
// (first m tiles) and C (next m), with X_AA = L_AA^{-1} and X_CC = L_CC^{-1}
// known from the previous level,
//   L^{-1} = [[X_AA, 0], [X_CA, X_CC]],  X_CA = -X_CC (L_CA X_AA),
// in two launches per level m = 1, 2, 4, ...: T = L_CA X_AA, then
// X_CA = -X_CC T, one workgroup per 64 x 64 output tile and at most m tile
// products each (the serial chain is 2 log2(kSG) launches instead of a
// forward substitution down the group).  T is parked in the upper triangle
// of G (tile (j, i) holds T_ij), which the last launch clears while it writes
// G's diagonal tiles and G^T.
// acc = sum_{k < nk} P_k Q_k over 64 x 64 tiles (row-major, leading
// dimensions from src), staged through LDS with the next pair's loads in
// flight during each product; wave w owns rows 16 w .. 16 w + 15.
template <class Src>
__device__ __forceinline__ void tile_gemm(double* sP, double* sQ, int nk, Src src, v4d* acc) {
  constexpr int NE = kNB * kNB / 256;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
  double vp[NE], vq[NE];
  auto gload = [&](int k) {
    const double *P, *Q;
    int64_t lp, lq;
    src(k, P, lp, Q, lq);
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      vp[it] = P[(int64_t)(e >> 6) * lp + (e & 63)];
      vq[it] = Q[(int64_t)(e >> 6) * lq + (e & 63)];
    }
  };
  if (nk > 0) gload(0);
  for (int k = 0; k < nk; ++k) {
    __syncthreads();   // the previous product has read sP and sQ
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int e = tid + 256 * it;
      sP[(e >> 6) * LDT + (e & 63)] = vp[it];
      sQ[(e >> 6) * LDT + (e & 63)] = vq[it];
    }
    if (k + 1 < nk) gload(k + 1);
    __syncthreads();
#pragma unroll 4
    for (int k0 = 0; k0 < kNB; k0 += 4) {
      const double a = sP[(16 * w + r16) * LDT + k0 + kq];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double b = sQ[(k0 + kq) * LDT + 16 * u + r16];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_trsv_ginv(const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ flags,
                                                   const int* __restrict__ st_sys,
                                                   const int* __restrict__ st_pre, int cnt,
                                                   const double* __restrict__ Lam,
                                                   const double* __restrict__ Linv, double* Ginv, int m,
                                                   int phase) {
  __shared__ double sP[kNB * LDT];
  __shared__ double sQ[kNB * LDT];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int per = kSG * m / 2;   // output tiles per group at this level
  const int q = t / per, rem = t % per;
  const int pair = rem / (m * m), o = rem % (m * m);
  const int A0 = 2 * m * pair, C0 = A0 + m;
  const int i = C0 + o / m, j = A0 + o % m;   // group-local tile indices
  const int p0 = kSG * q, nseg = min(sd.P, p0 + kSG) - p0;
  if (i >= nseg) return;
  const int64_t ld = sd.Kpad;
  const double* Lt = Lam + sd.loff + (int64_t)p0 * kNB * ld + (int64_t)p0 * kNB;   // L_qq
  const double* Li = Linv + sd.dgoff + (int64_t)p0 * kNB * kNB;
  double* G = Ginv + sd.gioff + (int64_t)q * 2 * kGS * kGS;
  auto gt = [&](int r, int c) { return G + (int64_t)r * kNB * kGS + (int64_t)c * kNB; };
  // X_rc of the current level's inputs: the stored diagonal inverses on the
  // diagonal, G below it
  auto xt = [&](int r, int c, const double*& p, int64_t& l) {
    if (r == c) {
      p = Li + (int64_t)r * kNB * kNB;
      l = kNB;
    } else {
      p = gt(r, c);
      l = kGS;
    }
  };
  v4d acc[4] = {};
  if (phase == 0) {
    // T_ij = sum_{k = j}^{A0 + m - 1} L_ik X_kj
    tile_gemm(sP, sQ, A0 + m - j, [&](int kk, const double*& P, int64_t& lp, const double*& Q, int64_t& lq) {
      const int k = j + kk;
      P = Lt + (int64_t)i * kNB * ld + (int64_t)k * kNB;
      lp = ld;
      xt(k, j, Q, lq);
    }, acc);
  } else {
    // X_ij = -sum_{k = C0}^{i} X_ik T_kj, T_kj parked at tile (j, k)
    tile_gemm(sP, sQ, i - C0 + 1, [&](int kk, const double*& P, int64_t& lp, const double*& Q, int64_t& lq) {
      const int k = C0 + kk;
      xt(i, k, P, lp);
      Q = gt(j, k);
      lq = kGS;
    }, acc);
  }
  double* out = phase == 0 ? gt(j, i) : gt(i, j);
  const double sg = phase == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(int64_t)(16 * w + 4 * e + kq) * kGS + 16 * u + r16] = sg * acc[u][e];
}

// Last step of G_q: diagonal tiles from the stored inverses, tiles above the
// diagonal cleared, and G^T; one workgroup per tile (i, j) of the group.
__global__ void __launch_bounds__(256) k_trsv_gfinish(const SysDesc* __restrict__ sys,
                                                      const int* __restrict__ flags,
                                                      const int* __restrict__ st_sys,
                                                      const int* __restrict__ st_pre, int cnt,
                                                      const double* __restrict__ Linv, double* Ginv) {
  __shared__ double sT[kNB * LDT];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int q = t / (kSG * kSG), i = (t / kSG) % kSG, j = t % kSG;
  const int p0 = kSG * q, nseg = min(sd.P, p0 + kSG) - p0;
  if (i >= nseg || j >= nseg) return;
  double* G = Ginv + sd.gioff + (int64_t)q * 2 * kGS * kGS;
  double* GT = G + (int64_t)kGS * kGS;
  double* gij = G + (int64_t)i * kNB * kGS + (int64_t)j * kNB;
  double* gtji = GT + (int64_t)j * kNB * kGS + (int64_t)i * kNB;
  const double* src = i == j ? Linv + sd.dgoff + (int64_t)(p0 + i) * kNB * kNB : gij;
  const int64_t ls = i == j ? kNB : kGS;
  const int tid = threadIdx.x;
  constexpr int NE = kNB * kNB / 256;
  double v[NE];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    v[it] = i >= j ? src[(int64_t)(e >> 6) * ls + (e & 63)] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    sT[(e >> 6) * LDT + (e & 63)] = v[it];
    if (i <= j) gij[(int64_t)(e >> 6) * kGS + (e & 63)] = v[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + 256 * it;
    gtji[(int64_t)(e >> 6) * kGS + (e & 63)] = sT[(e & 63) * LDT + (e >> 6)];
  }
}

// vout_q = M vin_q for group q, M = G_q (lower triangular; backward = 0) or
// G_q^T (upper triangular; backward = 1), rows of the group 16 per
// workgroup: wave w takes 4 rows, the lanes stride over the row's columns
// inside the triangle, and a wave reduction gives each entry.
// Apply part: z_q = G_q r_q (or x_q = G_q^T z_q), 16 rows per workgroup, the
// wave's four rows with every load in flight at once (row r of G_q, lower
// triangular, ends with its tile's last column; row r of G_q^T starts with
// its tile's first; columns outside read as zero).
__device__ __forceinline__ void gapply_part(double* sv, const SysDesc& sd, int t, const double* __restrict__ Ginv,
                                            const double* __restrict__ vin, double* vout, int q, int backward) {
  const int p0 = kSG * q, nv = (min(sd.P, p0 + kSG) - p0) * kNB;
  const int base = p0 * kNB;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int k = tid; k < kGS; k += 256) sv[k] = k < nv ? vin[sd.voff + base + k] : 0.0;
  const double* M = Ginv + sd.gioff + (int64_t)q * 2 * kGS * kGS + (backward ? (int64_t)kGS * kGS : 0);
  const int r0 = 16 * t + 4 * w;
  double g[4][kSG];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int r = r0 + m;
    const int c0 = backward ? (r & ~63) : 0, c1 = backward ? nv : (r | 63) + 1;
    const double* row = M + (int64_t)r * kGS;
#pragma unroll
    for (int it = 0; it < kSG; ++it) {
      const int c = 64 * it + lane;
      g[m][it] = (c >= c0 && c < c1) ? row[c] : 0.0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double v = 0.0;
#pragma unroll
    for (int it = 0; it < kSG; ++it) v += g[m][it] * sv[64 * it + lane];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) vout[sd.voff + base + r0 + m] = v;
  }
}

// Forward update part: r_i -= L_{i,q} z_q for 16 rows i from row tile r0t on
// (workgroup t takes rows r0t*64 + 16 t ..): one row per 16 lanes, 4
// columns per lane of each of the group's 64-column segments, all of the
// row's loads in flight at once.
__device__ __forceinline__ void gfwd_part(double* sz, const SysDesc& sd, int t, const double* __restrict__ Lam,
                                          const double* __restrict__ z, double* r, int q, int r0t) {
  const int64_t ld = sd.Kpad;
  const int p0 = kSG * q, nseg = min(sd.P, kSG * (q + 1)) - p0;
  const int base = p0 * kNB;
  const int tid = threadIdx.x, g = tid >> 4, j = tid & 15;
  for (int k = tid; k < kGS; k += 256) sz[k] = k < nseg * kNB ? z[sd.voff + base + k] : 0.0;
  const int i0 = r0t * kNB + 16 * t + g;
  const double* A = Lam + sd.loff + (int64_t)i0 * ld + base + 4 * j;
  double a[kSG][4];
#pragma unroll
  for (int sg = 0; sg < kSG; ++sg) {
    if (sg < nseg) {
      ld4(A + sg * kNB, a[sg]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[sg][u] = 0.0;
    }
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int sg = 0; sg < kSG; ++sg)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += a[sg][u] * sz[sg * kNB + 4 * j + u];
  const double v = gsum16(acc);
  if (j == 0) r[sd.voff + i0] -= v;
}

// Backward update part: z_c -= L_{q,c}^T x_q for the kBwdCW columns of
// column strip t (strips of kBwdCW columns from column tile c0t on, so that
// late groups, which have few column tiles to their left, still spread over
// many workgroups): 256 / kBwdCW row phases, each 16-lane row read one
// 128-byte line, 32 loads in flight per lane and batch; the phases' partial
// sums are added in a fixed order.
__device__ __forceinline__ void gbwd_part(double* sx, double* sp, const SysDesc& sd, int t,
                                          const double* __restrict__ Lam, const double* __restrict__ x, double* z,
                                          int q, int c0t) {
  constexpr int NRG = 256 / kBwdCW;
  const int64_t ld = sd.Kpad;
  const int p0 = kSG * q, nrow = (min(sd.P, kSG * (q + 1)) - p0) * kNB;
  const int base = p0 * kNB;
  const int tid = threadIdx.x, cc = tid % kBwdCW, rg = tid / kBwdCW;
  const int col0 = c0t * kNB + t * kBwdCW;
  for (int k = tid; k < kGS; k += 256) sx[k] = k < nrow ? x[sd.voff + base + k] : 0.0;
  __syncthreads();
  const double* A = Lam + sd.loff + (int64_t)base * ld + col0 + cc;
  double acc = 0.0;
  for (int r0 = 0; r0 < kGS; r0 += 32 * NRG) {
    double a[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int rr = r0 + rg + NRG * u;
      a[u] = rr < nrow ? A[(int64_t)rr * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) acc += a[u] * sx[r0 + rg + NRG * u];
  }
  sp[rg * kBwdCW + cc] = acc;
  __syncthreads();
  if (tid < kBwdCW) {
    double v = 0.0;
    for (int g = 0; g < NRG; ++g) v += sp[g * kBwdCW + tid];
    z[sd.voff + col0 + tid] -= v;
  }
}

__global__ void __launch_bounds__(256) k_trsv_gapply(const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags,
                                                     const int* __restrict__ st_sys,
                                                     const int* __restrict__ st_pre, int cnt,
                                                     const double* __restrict__ Ginv,
                                                     const double* __restrict__ vin, double* vout, int q,
                                                     int backward) {
  __shared__ double sv[kGS];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  gapply_part(sv, sd, blockIdx.x - st_pre[si], Ginv, vin, vout, q, backward);
}

__global__ void __launch_bounds__(256) k_trsv_gfwd(const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ flags,
                                                   const int* __restrict__ st_sys,
                                                   const int* __restrict__ st_pre, int cnt,
                                                   const double* __restrict__ Lam,
                                                   const double* __restrict__ z, double* r, int q) {
  __shared__ double sz[kGS];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  gfwd_part(sz, sd, blockIdx.x - st_pre[si], Lam, z, r, q, kSG * (q + 1));
}

__global__ void __launch_bounds__(256) k_trsv_gbwd(const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ flags,
                                                   const int* __restrict__ st_sys,
                                                   const int* __restrict__ st_pre, int cnt,
                                                   const double* __restrict__ Lam,
                                                   const double* __restrict__ x, double* z, int q) {
  __shared__ double sx[kGS];
  __shared__ double sp[256];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  gbwd_part(sx, sp, sd, blockIdx.x - st_pre[si], Lam, x, z, q, 0);
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

void launch_chol_update(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag,
                        double* Linv, const int* ssys, const int* spre, int cnt, int total, int p) {
  hipLaunchKernelGGL(k_chol_update, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, Linv, ssys,
                     spre, cnt, p);
}

void launch_chol_update_wide(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                             const int* ssys, const int* spre, int cnt, int total, int p, int mode) {
  if (total)
    hipLaunchKernelGGL(k_chol_update_wide, dim3(total), dim3(256), 0, st, sys, flags, Lam, ssys, spre,
                       cnt, p, mode);
}

void launch_chol_fused(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                       double* PB, const int* ssys, const int* spre, int cnt, int total, int p) {
  if (total)
    hipLaunchKernelGGL(k_chol_fused, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, Linv, PB, ssys, spre,
                       cnt, p);
}

void launch_chol_look(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                      const int* hsys, const int* hpre, int hcnt, int htot, const int* lsys, const int* lpre,
                      int lcnt, int ltot, int p) {
  if (htot + ltot)
    hipLaunchKernelGGL(k_chol_look, dim3(htot + ltot), dim3(256), 0, st, sys, flags, Lam, Ldiag, Linv, hsys, hpre,
                       hcnt, htot, lsys, lpre, lcnt, p);
}

void launch_chol_left(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag, double* Linv,
                      const int* ssys, const int* spre, int cnt, int total, int j) {
  if (total)
    hipLaunchKernelGGL(k_chol_left, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, Linv, ssys, spre, cnt, j);
}

void launch_trsv_ginv(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* Linv,
                      double* Ginv, int m, int phase) {
  if (total)
    hipLaunchKernelGGL(k_trsv_ginv, dim3(total), dim3(256), 0, st, sys, flags, ssys, spre, cnt, Lam, Linv, Ginv,
                       m, phase);
}

void launch_trsv_gfinish(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                         const int* spre, int cnt, int total, const double* Linv, double* Ginv) {
  if (total)
    hipLaunchKernelGGL(k_trsv_gfinish, dim3(total), dim3(256), 0, st, sys, flags, ssys, spre, cnt, Linv, Ginv);
}

void launch_trsv_gapply(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                        const int* spre, int cnt, int total, const double* Ginv, const double* vin,
                        double* vout, int q, int backward) {
  if (total)
    hipLaunchKernelGGL(k_trsv_gapply, dim3(total), dim3(256), 0, st, sys, flags, ssys, spre, cnt, Ginv, vin,
                       vout, q, backward);
}

void launch_trsv_gfwd(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* z, double* r,
                      int q) {
  if (total)
    hipLaunchKernelGGL(k_trsv_gfwd, dim3(total), dim3(256), 0, st, sys, flags, ssys, spre, cnt, Lam, z, r, q);
}

void launch_trsv_gbwd(hipStream_t st, const SysDesc* sys, const int* flags, const int* ssys,
                      const int* spre, int cnt, int total, const double* Lam, const double* x, double* z,
                      int q) {
  if (total)
    hipLaunchKernelGGL(k_trsv_gbwd, dim3(total), dim3(256), 0, st, sys, flags, ssys, spre, cnt, Lam, x, z, q);
}

void launch_trsv_small(hipStream_t st, int nsmall, const SysDesc* sys, const int* flags,
                       const int* small_ids, const double* Lam, const double* Linv,
                       const double* rhs, double* x) {
  if (nsmall)
    hipLaunchKernelGGL(k_trsv_small, dim3(nsmall), dim3(kSvT), 0, st, sys, flags, small_ids, Lam, Linv,
                       rhs, x);
}

}  // namespace psdp
