// Device routines shared by the kernels: workgroup-level dense kernels on
// one n x n block (n <= 128) with operands in global memory or LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace psdp {

// C = alpha op(A) op(B) + beta D for row-major n x n matrices (leading
// dimension n), on the 64 x 64 output tiles t = part, part + nparts, ... of
// the block (all of them for part 0 of 1; a grid that gives each block
// several workgroups passes blockIdx.y and gridDim.y).  256 threads; 4 x 4
// outputs per thread, inner dimension staged through LDS in chunks of 16.
// A and B must not alias C; D may alias C or be null.  sA and sB hold
// 16 * 64 doubles each.
__device__ inline void wg_gemm_part(int n, const double* __restrict__ A, int tA,
                                    const double* __restrict__ B, int tB, double* C, double alpha,
                                    const double* D, double beta, double* sA, double* sB, int part,
                                    int nparts) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int nt = (n + 63) / 64;
  for (int t = part; t < nt * nt; t += nparts) {
    const int i0 = 64 * (t / nt), j0 = 64 * (t % nt);
    {
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int k0 = 0; k0 < n; k0 += 16) {
        for (int e = tid; e < 1024; e += 256) {
          int kk, ii;
          if (tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          const int i = i0 + ii, k = k0 + kk;
          double v = 0.0;
          if (i < n && k < n) v = tA ? A[(int64_t)k * n + i] : A[(int64_t)i * n + k];
          sA[kk * 64 + ii] = v;
          int jj, kb;
          if (tB) { kb = e & 15; jj = e >> 4; } else { jj = e & 63; kb = e >> 6; }
          const int j = j0 + jj, k2 = k0 + kb;
          double w = 0.0;
          if (j < n && k2 < n) w = tB ? B[(int64_t)j * n + k2] : B[(int64_t)k2 * n + j];
          sB[kb * 64 + jj] = w;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
          double a[4], b[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = sA[kk * 64 + ty * 4 + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = sB[kk * 64 + tx * 4 + c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + ty * 4 + r;
        if (i >= n) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = j0 + tx * 4 + c;
          if (j >= n) continue;
          double v = alpha * acc[r][c];
          if (D) v += beta * D[(int64_t)i * n + j];
          C[(int64_t)i * n + j] = v;
        }
      }
    }
  }
}

// the whole block in one workgroup
__device__ inline void wg_gemm(int n, const double* __restrict__ A, int tA,
                               const double* __restrict__ B, int tB, double* C, double alpha,
                               const double* D, double beta, double* sA, double* sB) {
  wg_gemm_part(n, A, tA, B, tB, C, alpha, D, beta, sA, sB, 0, 1);
}

// 1/sqrt(d) for a positive finite d: the hardware estimate refined by two
// Newton steps for the inverse square root, y += y (1 - d y^2) / 2.
__device__ inline double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int i = 0; i < 2; ++i) y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
  return y;
}

// value of v in lane l (l uniform) for every lane
__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The dispatcher hands consecutive workgroups to the device's eight XCDs in
// turn.  xcd_order(b, total) renumbers workgroup b of a grid of total so
// that each XCD receives one contiguous range of [0, total): neighbouring
// work items, which read the same operands, then share one XCD's L2.
constexpr int kXCD = 8;
__device__ __forceinline__ int xcd_order(int b, int total) {
  const int per = total / kXCD, rem = total % kXCD, x = b % kXCD;
  return x * per + min(x, rem) + b / kXCD;
}

// value of v in lane C of each row of 16 lanes, for every lane of that row
// (one 64-bit DPP row_newbcast move; no LDS).  Every lane of the row must
// be active.
template <int C>
__device__ __forceinline__ double row_bcast16(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, false);
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

// Whether the Cholesky factorisation of the symmetric 16 x 16 matrix held by
// a row of 16 lanes succeeds (every pivot positive and finite): lane r holds
// row r in a (only the lower triangle is read; a is overwritten).  Column k
// is scaled by the Newton reciprocal square root of its pivot and values
// travel by DPP row broadcasts; the result is the same on the row's 16 lanes.
__device__ __forceinline__ bool rows_chol_ok16(double* a, int r) {
  bool bad = false;
  static_for<16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double d = row_bcast16<k>(a[k]);
    const bool bb = !(d > 0.0) || !isfinite(d);
    bad = bad || bb;
    d = bb ? 1.0 : d;
    const double rs = rsqrt_nr(d);
    const double lrk = a[k] * rs;   // L[r][k] on the lanes r >= k that use it
    static_for<16>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c > k) {
        const double lck = row_bcast16<c>(lrk);
        a[c] = r >= c ? a[c] - lrk * lck : a[c];
      }
    });
  });
  return !bad;
}

// In-place lower Cholesky of the n x n matrix in LDS (leading dimension ld).
// Reads only the lower triangle.  A pivot that is not a positive finite
// number marks failure (*fail = 1) and is replaced by 1 so the sweep stays
// finite.  All threads of the workgroup must call it.
__device__ inline void wg_potrf(double* A, int n, int ld, int* fail) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      double d = A[k * ld + k];
      if (!(d > 0.0) || !isfinite(d)) {
        *fail = 1;
        d = 1.0;
      }
      A[k * ld + k] = sqrt(d);
    }
    __syncthreads();
    const double piv = A[k * ld + k];
    for (int i = k + 1 + tid; i < n; i += nt) A[i * ld + k] = A[i * ld + k] / piv;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += nt) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) A[i * ld + j] -= A[i * ld + k] * A[j * ld + k];
    }
    __syncthreads();
  }
}

// In-place inverse of the lower triangular matrix in LDS (column sweep from
// the last column, as in the unblocked LAPACK inverse).  Needs n <= blockDim.
__device__ inline void wg_trtri_lower(double* A, int n, int ld) {
  const int tid = threadIdx.x;
  for (int j = n - 1; j >= 0; --j) {
    if (tid == 0) A[j * ld + j] = 1.0 / A[j * ld + j];
    __syncthreads();
    const double ajj = -A[j * ld + j];
    const int i = j + 1 + tid;
    double v = 0.0;
    if (i < n) {
      for (int k = j + 1; k <= i; ++k) v += A[i * ld + k] * A[k * ld + j];
      v *= ajj;
    }
    __syncthreads();
    if (i < n) A[i * ld + j] = v;
    __syncthreads();
  }
}

__device__ inline int find_owner(const int* prefix, int count, int x) {
  // largest s in [0, count) with prefix[s] <= x (prefix[0] = 0, increasing)
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace psdp
