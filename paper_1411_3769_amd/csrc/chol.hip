// Dense FP64 Cholesky of the Schur complement and the two triangular solves
// (Alg. 2, root steps 1 and 2: Lambda dy = Omega).  The paper factors Lambda
// on a root processor with LAPACK; here every system of a batch is factored
// together, tile by tile.
//
// Storage: each system's Kpad x Kpad matrix is row-major (leading dimension
// Kpad, a multiple of 64); rows/columns past K hold the identity, so the
// factor of the padded matrix is blockdiag(L, I) and no kernel needs ragged
// edges.  The off-diagonal tiles of the factor overwrite the lower triangle;
// the factored diagonal tiles go to a separate array Ldiag[P][64][64] (other
// workgroups of the same step still read the unfactored diagonal tile); the
// strict upper triangle keeps Lambda.
//
// Right-looking blocked algorithm, step p (panel column p):
//   panel  : every workgroup loads the 64 x 64 diagonal tile, factors it in
//            LDS (redundantly: this replaces a separate launch), then either
//            writes L_pp back (tile row p) or solves L_ip = A_ip L_pp^{-T}
//            for one tile row below it;
//   update : every tile (i, j), p < j <= i, gets A_ij -= L_ip L_jp^T.
// Steps are launched for the whole batch; a (step, system) table maps
// workgroups to systems.
#include <hip/hip_runtime.h>

#include "devcommon.h"
#include "internal.h"

namespace psdp {

constexpr int LDT = kNB + 1;   // LDS leading dimension of a 64 x 64 tile

__device__ inline void load_tile_lower(double* s, const double* A, int64_t ld) {
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) {
    const int r = e / kNB, c = e % kNB;
    s[r * LDT + c] = A[r * ld + c];
  }
}

__global__ void __launch_bounds__(256) k_chol_panel(const SysDesc* __restrict__ sys, int* flags,
                                                    double* Lam, double* Ldiag,
                                                    const int* __restrict__ st_sys,
                                                    const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sL[kNB * LDT];
  __shared__ double sA[kNB * LDT];
  __shared__ int fl;
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  const int tid = threadIdx.x;
  if (tid == 0) fl = 0;
  load_tile_lower(sL, A + (int64_t)p * kNB * ld + (int64_t)p * kNB, ld);
  __syncthreads();
  wg_potrf(sL, kNB, LDT, &fl);
  if (t == 0) {
    double* D = Ldiag + sd.dgoff + (int64_t)p * kNB * kNB;
    for (int e = tid; e < kNB * kNB; e += blockDim.x) {
      const int r = e / kNB, c = e % kNB;
      D[e] = c <= r ? sL[r * LDT + c] : 0.0;
    }
    if (tid == 0 && fl) atomicOr(&flags[s], F_LAMFAIL);
    return;
  }
  const int i = p + t;
  double* Ai = A + (int64_t)i * kNB * ld + (int64_t)p * kNB;
  for (int e = tid; e < kNB * kNB; e += blockDim.x) {
    const int r = e / kNB, c = e % kNB;
    sA[r * LDT + c] = Ai[(int64_t)r * ld + c];
  }
  __syncthreads();
  // row r of X solves x L_pp^T = a, i.e. L_pp x^T = a^T: forward
  // substitution, four lanes per row splitting the inner products.
  const int r = tid >> 2, q = tid & 3;
  double xr[kNB / 4];
#pragma unroll
  for (int c = 0; c < kNB; ++c) {
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < c; ++k)
      if ((k & 3) == q) part += xr[k >> 2] * sL[c * LDT + k];
    part += __shfl_xor(part, 1, 4);
    part += __shfl_xor(part, 2, 4);
    const double xc = (sA[r * LDT + c] - part) / sL[c * LDT + c];
    if ((c & 3) == q) xr[c >> 2] = xc;
  }
#pragma unroll
  for (int k = 0; k < kNB / 4; ++k) Ai[(int64_t)r * ld + k * 4 + q] = xr[k];
}

// A_ij -= L_ip L_jp^T for every tile p < j <= i; 4 x 4 outputs per thread,
// the inner dimension (64) staged through LDS in chunks of 16.
__global__ void __launch_bounds__(256) k_chol_update(const SysDesc* __restrict__ sys,
                                                     const int* __restrict__ flags, double* Lam,
                                                     const int* __restrict__ st_sys,
                                                     const int* __restrict__ st_pre, int cnt,
                                                     int p) {
  __shared__ double sa[16 * 64];
  __shared__ double sb[16 * 64];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_CHOLSEL)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  double* A = Lam + sd.loff;
  // triangular index t -> (ii >= jj)
  int ii = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  const int jj = t - ii * (ii + 1) / 2;
  const int i = p + 1 + ii, j = p + 1 + jj;
  const double* Li = A + (int64_t)i * kNB * ld + (int64_t)p * kNB;
  const double* Lj = A + (int64_t)j * kNB * ld + (int64_t)p * kNB;
  double* C = A + (int64_t)i * kNB * ld + (int64_t)j * kNB;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < kNB; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int kk = e & 15, rr = e >> 4;
      sa[kk * 64 + rr] = Li[(int64_t)rr * ld + k0 + kk];
      sb[kk * 64 + rr] = Lj[(int64_t)rr * ld + k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = sa[kk * 64 + ty * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = sb[kk * 64 + tx * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int rr = ty * 4 + u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cc = tx * 4 + v;
      if (i != j || cc <= rr) C[(int64_t)rr * ld + cc] -= acc[u][v];
    }
  }
}

// wave-level solve of L x = b (lower, 64 x 64 in LDS) by lane-parallel
// inner products; every lane ends with x[lane].
__device__ inline double wave_fwd(const double* sL, double b_lane) {
  const int lane = threadIdx.x & 63;
  double x = 0.0;
  for (int c = 0; c < kNB; ++c) {
    double part = lane < c ? x * sL[c * LDT + lane] : 0.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
    const double bc = __shfl(b_lane, c, 64);
    const double xc = (bc - part) / sL[c * LDT + c];
    if (lane == c) x = xc;
  }
  return x;
}

// wave-level solve of L^T x = b.
__device__ inline double wave_bwd(const double* sL, double b_lane) {
  const int lane = threadIdx.x & 63;
  double x = 0.0;
  for (int c = kNB - 1; c >= 0; --c) {
    double part = lane > c ? sL[lane * LDT + c] * x : 0.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
    const double bc = __shfl(b_lane, c, 64);
    const double xc = (bc - part) / sL[c * LDT + c];
    if (lane == c) x = xc;
  }
  return x;
}

// forward step p: z_p = L_pp^{-1} r_p (tile 0 writes it); tiles i > p update
// r_i -= L_ip z_p.
__device__ inline void load_diag(double* s, const double* D) {
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) s[(e / kNB) * LDT + e % kNB] = D[e];
}

__global__ void __launch_bounds__(256) k_trsv_fwd(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ Lam,
                                                  const double* __restrict__ Ldiag, double* r,
                                                  double* z, const int* __restrict__ st_sys,
                                                  const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sL[kNB * LDT];
  __shared__ double sx[kNB];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int t = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  const int64_t ld = sd.Kpad;
  const double* A = Lam + sd.loff;
  double* rs = r + sd.voff;
  double* zs = z + sd.voff;
  load_diag(sL, Ldiag + sd.dgoff + (int64_t)p * kNB * kNB);
  __syncthreads();
  if (threadIdx.x < 64) {
    const double x = wave_fwd(sL, rs[p * kNB + threadIdx.x]);
    sx[threadIdx.x] = x;
    if (t == 0) zs[p * kNB + threadIdx.x] = x;
  }
  __syncthreads();
  if (t == 0) return;
  const int i = p + t;
  const double* Li = A + (int64_t)i * kNB * ld + (int64_t)p * kNB;
  const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
  double part = 0.0;
  for (int c = q; c < kNB; c += 4) part += Li[(int64_t)row * ld + c] * sx[c];
  part += __shfl_xor(part, 1, 4);
  part += __shfl_xor(part, 2, 4);
  if (q == 0) rs[i * kNB + row] -= part;
}

// backward step p: x_p = L_pp^{-T} z_p (tile p writes it); tiles i < p
// update z_i -= L_pi^T x_p.
__global__ void __launch_bounds__(256) k_trsv_bwd(const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ flags,
                                                  const double* __restrict__ Lam,
                                                  const double* __restrict__ Ldiag, double* z,
                                                  double* x, const int* __restrict__ st_sys,
                                                  const int* __restrict__ st_pre, int cnt, int p) {
  __shared__ double sL[kNB * LDT];
  __shared__ double sx[kNB];
  const int si = find_owner(st_pre, cnt, blockIdx.x);
  const int s = st_sys[si];
  const int i = blockIdx.x - st_pre[si];
  if (!(flags[s] & F_ACTIVE)) return;
  const SysDesc sd = sys[s];
  if (p >= sd.P) return;
  const int64_t ld = sd.Kpad;
  const double* A = Lam + sd.loff;
  double* zs = z + sd.voff;
  double* xs = x + sd.voff;
  load_diag(sL, Ldiag + sd.dgoff + (int64_t)p * kNB * kNB);
  __syncthreads();
  if (threadIdx.x < 64) {
    const double v = wave_bwd(sL, zs[p * kNB + threadIdx.x]);
    sx[threadIdx.x] = v;
    if (i == p) xs[p * kNB + threadIdx.x] = v;
  }
  __syncthreads();
  if (i == p) return;
  const double* Lpi = A + (int64_t)p * kNB * ld + (int64_t)i * kNB;
  const int col = threadIdx.x >> 2, q = threadIdx.x & 3;
  double part = 0.0;
  for (int c = q; c < kNB; c += 4) part += Lpi[(int64_t)c * ld + col] * sx[c];
  part += __shfl_xor(part, 1, 4);
  part += __shfl_xor(part, 2, 4);
  if (q == 0) zs[i * kNB + col] -= part;
}

// launch wrappers --------------------------------------------------------------

void launch_chol_panel(hipStream_t st, const SysDesc* sys, int* flags, double* Lam, double* Ldiag,
                       const int* ssys, const int* spre, int cnt, int total, int p) {
  hipLaunchKernelGGL(k_chol_panel, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, ssys, spre, cnt, p);
}

void launch_chol_update(hipStream_t st, const SysDesc* sys, const int* flags, double* Lam,
                        const int* ssys, const int* spre, int cnt, int total, int p) {
  hipLaunchKernelGGL(k_chol_update, dim3(total), dim3(256), 0, st, sys, flags, Lam, ssys, spre, cnt, p);
}

void launch_trsv_fwd(hipStream_t st, const SysDesc* sys, const int* flags, const double* Lam,
                     const double* Ldiag, double* r, double* z, const int* ssys, const int* spre,
                     int cnt, int total, int p) {
  hipLaunchKernelGGL(k_trsv_fwd, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, r, z, ssys, spre, cnt, p);
}

void launch_trsv_bwd(hipStream_t st, const SysDesc* sys, const int* flags, const double* Lam,
                     const double* Ldiag, double* z, double* x, const int* ssys, const int* spre,
                     int cnt, int total, int p) {
  hipLaunchKernelGGL(k_trsv_bwd, dim3(total), dim3(256), 0, st, sys, flags, Lam, Ldiag, z, x, ssys, spre, cnt, p);
}

}  // namespace psdp
