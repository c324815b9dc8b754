// Polya set-up (Section III-A/B, Alg. 1) and the handle-level C ABI.
//
// The paper computes beta and H by d1 and d2 rounds of a neighbour-sum
// recursion (eq. beta, eq. H), distributed over MPI ranks.  Both recursions
// add the coefficients of (sum alpha) repeatedly, so after d rounds the
// weight of a shift delta is the multinomial coefficient d!/delta!.  On the
// GPU every coefficient is therefore independent: one thread per (h, gamma)
// for beta and one workgroup per (gamma, h) for H, with exact int64 integer
// arithmetic (degrees <= 20) and H folded over lambda in ascending order with
// separate multiply and add (this file is compiled without FP contraction).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace psdp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

__constant__ int64_t c_fact[kMaxDeg + 1];

static int64_t host_fact(int d) {
  int64_t f = 1;
  for (int i = 2; i <= d; ++i) f *= i;
  return f;
}

static int64_t binom(int a, int b) {
  if (b < 0 || b > a) return 0;
  double r = 1;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return (int64_t)llround(r);
}

// W_d in descending lexicographic order (Notation): alpha_1^d first.
static void monomials(int l, int d, std::vector<int>& out) {
  out.clear();
  std::vector<int> cur(l, 0);
  // recursive enumeration with the first entry descending
  struct Rec {
    static void go(int l, int pos, int rem, std::vector<int>& cur, std::vector<int>& out) {
      if (pos == l - 1) {
        cur[pos] = rem;
        out.insert(out.end(), cur.begin(), cur.end());
        return;
      }
      for (int v = rem; v >= 0; --v) {
        cur[pos] = v;
        go(l, pos + 1, rem - v, cur, out);
      }
    }
  };
  Rec::go(l, 0, d, cur, out);
}

BasisInfo make_basis(int n) {
  BasisInfo b;
  b.n = n;
  b.NG = (n + kTB - 1) / kTB;
  for (int g1 = 0; g1 < b.NG; ++g1) {
    for (int g2 = g1; g2 < b.NG; ++g2) {
      b.gp_g1.push_back(g1);
      b.gp_g2.push_back(g2);
      b.gp_off.push_back((int)(b.pairs.size() / 2));
      const int p0 = g1 * kTB, p1 = std::min(n, p0 + kTB);
      const int q0 = g2 * kTB, q1 = std::min(n, q0 + kTB);
      for (int p = p0; p < p1; ++p)
        for (int q = q0; q < q1; ++q) {
          if (g1 == g2 && q < p) continue;
          b.pairs.push_back(p);
          b.pairs.push_back(q);
        }
      b.gp_size.push_back((int)(b.pairs.size() / 2) - b.gp_off.back());
    }
  }
  b.ngp = (int)b.gp_g1.size();
  return b;
}

// ---------------------------------------------------------------------------
// kernels (H1)
// ---------------------------------------------------------------------------

// d! / prod delta_i! by successive exact divisions (each partial quotient is
// an integer because the remaining denominators divide the remaining
// numerator).
__device__ inline int64_t dev_multinomial(int d, const int* delta, int l) {
  int64_t r = c_fact[d];
  for (int i = 0; i < l; ++i) r /= c_fact[delta[i]];
  return r;
}

__global__ void k_beta(const int* __restrict__ Wp, const int* __restrict__ WL, int l, int L0, int L,
                       int d1, int64_t* __restrict__ beta, double* __restrict__ betaf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L0 * L) return;
  const int h = t / L, j = t % L;
  int delta[32];
  bool ok = true;
  for (int i = 0; i < l; ++i) {
    delta[i] = WL[j * l + i] - Wp[h * l + i];
    ok = ok && delta[i] >= 0;
  }
  const int64_t v = ok ? dev_multinomial(d1, delta, l) : 0;
  beta[t] = v;
  betaf[t] = (double)v;
}

// one workgroup per (m, h): integer weights c[h][m][lam] into LDS, then
// H[m][h] = sum_lam c * A_lam entrywise.
__global__ void k_coef_H(const int* __restrict__ Wp, const int* __restrict__ WM,
                         const int* __restrict__ Wa, int l, int L0, int M, int Na, int n, int d2,
                         const double* __restrict__ A, int64_t* __restrict__ coef,
                         double* __restrict__ H) {
  extern __shared__ int64_t s_c[];
  const int m = blockIdx.x / L0, h = blockIdx.x % L0;
  for (int lam = threadIdx.x; lam < Na; lam += blockDim.x) {
    int delta[32];
    bool ok = true;
    for (int i = 0; i < l; ++i) {
      delta[i] = WM[m * l + i] - Wp[h * l + i] - Wa[lam * l + i];
      ok = ok && delta[i] >= 0;
    }
    const int64_t v = ok ? dev_multinomial(d2, delta, l) : 0;
    s_c[lam] = v;
    coef[((int64_t)h * M + m) * Na + lam] = v;
  }
  __syncthreads();
  const int nn = n * n;
  double* out = H + ((int64_t)m * L0 + h) * nn;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    double acc = 0.0;
    for (int lam = 0; lam < Na; ++lam) {
      const int64_t c = s_c[lam];
      if (c != 0) acc = acc + (double)c * A[(int64_t)lam * nn + e];
    }
    out[e] = acc;
  }
}

// *bad = 1 if any of the n values is not finite (one workgroup)
__global__ void k_nonfinite(const double* __restrict__ v, int64_t n, double* bad) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mine |= !isfinite(v[i]);
  if (mine) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) *bad = any ? 1.0 : 0.0;
}

__global__ void k_scale(const int* __restrict__ Wp, const int* __restrict__ WL,
                        const int* __restrict__ WM, int l, int L0, int L, int M, int dp,
                        int dM, const int64_t* __restrict__ beta, double delta, double eps,
                        double* __restrict__ scale, double* __restrict__ cdiag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L + M) return;
  if (j < L) {
    // eq. Cj: s_j = sum_h beta_{h,j} dp!/h!
    int64_t s = 0;
    for (int h = 0; h < L0; ++h) s += beta[h * L + j] * dev_multinomial(dp, Wp + h * l, l);
    scale[j] = (double)s;
    cdiag[j] = delta * (double)s;
  } else {
    const int64_t s = dev_multinomial(dM, WM + (j - L) * l, l);
    scale[j] = (double)s;
    cdiag[j] = eps * (double)s;
  }
}

}  // namespace psdp

using namespace psdp;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void psdp_setup_opts_default(psdp_setup_opts* o) {
  if (!o) return;
  o->da = 1;
  o->d1 = -1;
  o->d2 = -1;
  o->delta = 1e-3;
  o->eps = 1e-3;
  o->paper_literal = 0;
  o->a_on_device = 0;
}

void psdp_opts_default(psdp_opts* o) {
  if (!o) return;
  o->gap_tol = 1e-8;
  o->feas_tol = 1e-8;
  o->max_iter = 100;
  o->sigma = 1.0 / 3.0;
  o->step_frac = 0.95;
  o->ladder_rho = 0.9;
  o->ladder_len = 300;
  o->verdict_mode = PSDP_VERDICT_PAPER_THEN_PHASE1;
  o->precision = PSDP_PREC_FP64;
  o->ir_max = -1;
  o->stream = nullptr;
  o->record_history = 0;
  o->prof = nullptr;
  o->warm_y = nullptr;
  o->warm_logx = nullptr;
  o->warm_iter_cap = 0;
  o->warm_margin = 1e-6;
  o->warm_center = 1;
  o->asm_path = -1;
  o->solve_path = -1;
  o->use_graph = 1;
  o->label_gap = 0.0;
}

const char* psdp_last_error(void) { return g_err.c_str(); }

const char* psdp_version(void) { return "polyaipm 0.1 (gfx950)"; }

// Set-up of one system up to its kernels, all asynchronous on the null
// stream; *rb receives the device address of its read-back region (betaf,
// scale, cdiag, non-finite flag of A: *nrb doubles), which setup_finish
// parses once the stream has drained.
static int setup_begin(const double* A, int n, int l, int dp, int d, const psdp_setup_opts* o,
                       psdp_sdp** out, const double** rb_dev, int64_t* nrb_out) {
  try {
    if (!out) return fail(PSDP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A) return fail(PSDP_EINVAL, "A is NULL");
    psdp_setup_opts opt;
    psdp_setup_opts_default(&opt);
    if (o) opt = *o;
    const int da = opt.da;
    const int d1 = opt.d1 >= 0 ? opt.d1 : d;
    const int d2 = opt.d2 >= 0 ? opt.d2 : d;
    if (n < 1 || n > kMaxN) return fail(PSDP_EINVAL, "n must be in [1, 128]");
    if (l < 1 || l > 32) return fail(PSDP_EINVAL, "l must be in [1, 32]");
    if (dp < 0 || da < 1 || d1 < 0 || d2 < 0) return fail(PSDP_EINVAL, "negative degree");
    if (!(opt.delta > 0.0) || !(opt.eps >= 0.0) || !std::isfinite(opt.delta) ||
        !std::isfinite(opt.eps))
      return fail(PSDP_EINVAL, "delta must be > 0 and eps >= 0");
    if (dp + d1 > kMaxDeg || dp + da + d2 > kMaxDeg)
      return fail(PSDP_EOVERFLOW, "Polya degree above 20: multinomials exceed int64");
    const int64_t L0 = binom(l + dp - 1, l - 1), L = binom(l + dp + d1 - 1, l - 1);
    const int64_t M = binom(l + dp + da + d2 - 1, l - 1), Na = binom(l + da - 1, l - 1);
    const int64_t Nt = (int64_t)n * (n + 1) / 2;
    const int64_t K = L0 * Nt;
    if (L0 > 100000 || L > 10000000 || M > 10000000 || Na > 4096 || K > 200000)
      return fail(PSDP_EOVERFLOW, "problem dimensions too large");
    if (!opt.a_on_device) {
      for (int64_t i = 0; i < Na * n * n; ++i)
        if (!std::isfinite(A[i])) return fail(PSDP_EINVAL, "A has a non-finite entry");
    }
    int dev = 0;
    PSDP_HIP(hipGetDevice(&dev));

    psdp_sdp* s = new psdp_sdp();
    s->n = n; s->l = l; s->da = da; s->dp = dp; s->d1 = d1; s->d2 = d2;
    s->L0 = (int)L0; s->L = (int)L; s->M = (int)M; s->Na = (int)Na; s->Nt = (int)Nt;
    s->nb = (int)(L + M);
    s->K = K;
    s->Kpad = round_up(K, kNB);
    s->delta = opt.delta;
    s->eps = opt.paper_literal ? 0.0 : opt.eps;
    s->paper_literal = opt.paper_literal;
    s->device = dev;
    monomials(l, dp, s->Wp);
    monomials(l, dp + d1, s->WL);
    monomials(l, dp + da + d2, s->WM);
    monomials(l, da, s->Wa);
    s->bmask.assign(L0 * L, 0);
    for (int h = 0; h < L0; ++h)
      for (int j = 0; j < L; ++j) {
        bool ge = true;
        for (int i = 0; i < l; ++i) ge = ge && s->WL[j * l + i] >= s->Wp[h * l + i];
        s->bmask[h * L + j] = ge;
      }
    s->hmask.assign(M * L0, 0);
    for (int m = 0; m < M; ++m)
      for (int h = 0; h < L0; ++h) {
        bool ge = true;
        for (int i = 0; i < l; ++i) ge = ge && s->WM[m * l + i] >= s->Wp[h * l + i];
        s->hmask[m * L0 + h] = ge;
      }
    s->basis = make_basis(n);

    // one device allocation for the handle
    const int64_t nn = (int64_t)n * n;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off += (bytes + 255) / 256 * 256; return r; };
    const size_t oA = take(Na * nn * 8), oB = take(L0 * L * 8), oC = take(L0 * M * Na * 8);
    const size_t oH = take(M * L0 * nn * 8);
    // read-back region, contiguous: betaf, scale, cdiag, non-finite flag of A
    const int64_t nrb = L0 * L + 2 * (L + M) + 1;
    const size_t oRb = take(nrb * 8);
    const size_t oBf = oRb, oS = oRb + L0 * L * 8, oCd = oS + (L + M) * 8, oBad = oCd + (L + M) * 8;
    // integer tables, contiguous: basis, Wp, WL, WM, Wa
    std::vector<int> tab;
    tab.insert(tab.end(), s->basis.pairs.begin(), s->basis.pairs.end());
    const size_t iWp = tab.size();
    tab.insert(tab.end(), s->Wp.begin(), s->Wp.end());
    const size_t iWL = tab.size();
    tab.insert(tab.end(), s->WL.begin(), s->WL.end());
    const size_t iWM = tab.size();
    tab.insert(tab.end(), s->WM.begin(), s->WM.end());
    const size_t iWa = tab.size();
    tab.insert(tab.end(), s->Wa.begin(), s->Wa.end());
    const size_t oBa = take(tab.size() * 4);
    const size_t oWp = oBa + iWp * 4, oWL = oBa + iWL * 4, oWM = oBa + iWM * 4, oWa = oBa + iWa * 4;
    s->dbytes = off;
    if (hipMalloc(&s->dmem, off) != hipSuccess) {
      delete s;
      return fail(PSDP_ENOMEM, "device allocation for the set-up failed");
    }
    char* base = (char*)s->dmem;
    s->dA = (double*)(base + oA);
    s->dbeta = (int64_t*)(base + oB);
    s->dcoef = (int64_t*)(base + oC);
    s->dH = (double*)(base + oH);
    s->dbetaf = (double*)(base + oBf);
    s->dscale = (double*)(base + oS);
    s->dcdiag = (double*)(base + oCd);
    s->dbasis = (int*)(base + oBa);
    int* dWp = (int*)(base + oWp);
    int* dWL = (int*)(base + oWL);
    int* dWM = (int*)(base + oWM);
    int* dWa = (int*)(base + oWa);

    int64_t fact[kMaxDeg + 1];
    for (int i = 0; i <= kMaxDeg; ++i) fact[i] = host_fact(i);
    auto cleanup = [&](int code, const std::string& msg) {
      hipFree(s->dmem);
      delete s;
      return fail(code, msg);
    };
    // the factorial table goes to constant memory once per device
    static bool fact_done[64] = {false};
    if (dev < 0 || dev >= 64) return cleanup(PSDP_EDEVICE, "device index out of range");
    if (!fact_done[dev]) {
      if (hipMemcpyToSymbol(HIP_SYMBOL(c_fact), fact, sizeof(fact)) != hipSuccess)
        return cleanup(PSDP_EDEVICE, "copy of the factorial table failed");
      fact_done[dev] = true;
    }
    hipError_t e = hipSuccess;
    e = hipMemcpyAsync(s->dA, A, Na * nn * 8,
                       opt.a_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(s->dbasis, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, 0);
    if (e != hipSuccess) return cleanup(PSDP_EDEVICE, std::string("set-up copy: ") + hipGetErrorString(e));

    {
      const int nt = (int)(L0 * L);
      hipLaunchKernelGGL(k_beta, dim3((nt + 255) / 256), dim3(256), 0, 0, dWp, dWL, l, (int)L0,
                         (int)L, d1, s->dbeta, s->dbetaf);
      hipLaunchKernelGGL(k_coef_H, dim3((unsigned)(M * L0)), dim3(256), Na * 8, 0, dWp, dWM, dWa, l,
                         (int)L0, (int)M, (int)Na, n, d2, s->dA, s->dcoef, s->dH);
      const int nbk = (int)(L + M);
      hipLaunchKernelGGL(k_scale, dim3((nbk + 255) / 256), dim3(256), 0, 0, dWp, dWL, dWM, l,
                         (int)L0, (int)L, (int)M, dp, dp + da + d2, s->dbeta, s->delta, s->eps,
                         s->dscale, s->dcdiag);
      double* dbad = (double*)(base + oBad);
      hipLaunchKernelGGL(k_nonfinite, dim3(1), dim3(256), 0, 0, s->dA, Na * nn, dbad);
      e = hipGetLastError();
      if (e != hipSuccess) return cleanup(PSDP_EDEVICE, std::string("set-up kernels: ") + hipGetErrorString(e));
    }
    *rb_dev = s->dbetaf;
    *nrb_out = nrb;
    *out = s;
    return PSDP_OK;
  } catch (const std::bad_alloc&) {
    return fail(PSDP_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(PSDP_EINVAL, "unexpected exception in psdp_polya_setup");
  }
}

// Parse the read-back of a begun set-up (host copy rb); on a non-finite A the
// handle is released and *out cleared.
static int setup_finish(psdp_sdp** out, const double* rb, int64_t nrb) {
  psdp_sdp* s = *out;
  if (rb[nrb - 1] != 0.0) {
    hipFree(s->dmem);
    delete s;
    *out = nullptr;
    return fail(PSDP_EINVAL, "A has a non-finite entry");
  }
  const int64_t L0 = s->L0, L = s->L, M = s->M;
  s->betaf.assign(rb, rb + L0 * L);
  s->scale_h.assign(rb + L0 * L, rb + L0 * L + (L + M));
  s->cdiag_h.assign(rb + L0 * L + (L + M), rb + L0 * L + 2 * (L + M));
  return PSDP_OK;
}

int psdp_polya_setup(const double* A, int n, int l, int dp, int d, const psdp_setup_opts* o,
                     psdp_sdp** out) {
  const double* rb_dev = nullptr;
  int64_t nrb = 0;
  int rc = setup_begin(A, n, l, dp, d, o, out, &rb_dev, &nrb);
  if (rc) return rc;
  try {
    // one read-back (it also waits for the kernels)
    std::vector<double> rb(nrb);
    const hipError_t e = hipMemcpy(rb.data(), rb_dev, nrb * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      psdp_free(*out);
      *out = nullptr;
      return fail(PSDP_EDEVICE, std::string("set-up read-back: ") + hipGetErrorString(e));
    }
    return setup_finish(out, rb.data(), nrb);
  } catch (const std::bad_alloc&) {
    psdp_free(*out);
    *out = nullptr;
    return fail(PSDP_ENOMEM, "host allocation failed");
  }
}

int psdp_polya_setup_batched(int count, const double* const* A, const int* n, const int* l,
                             const int* dp, const int* d, const psdp_setup_opts* o, psdp_sdp** out) {
  if (count < 0) return fail(PSDP_EINVAL, "count is negative");
  if (count > 0 && (!A || !n || !l || !dp || !d || !out)) return fail(PSDP_EINVAL, "NULL argument");
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  std::vector<const double*> rb_dev(count, nullptr);
  std::vector<int64_t> nrb(count, 0), roff(count + 1, 0);
  auto release = [&]() {
    for (int i = 0; i < count; ++i) {
      if (out[i]) psdp_free(out[i]);
      out[i] = nullptr;
    }
  };
  for (int i = 0; i < count; ++i) {
    const int rc = setup_begin(A[i], n[i], l[i], dp[i], d[i], o, &out[i], &rb_dev[i], &nrb[i]);
    if (rc) {
      const std::string msg = "system " + std::to_string(i) + ": " + psdp_last_error();
      release();
      return fail(rc, msg);
    }
    roff[i + 1] = roff[i] + nrb[i];
  }
  if (count == 0) return PSDP_OK;
  // every read-back into one pinned buffer, one wait
  double* host = nullptr;
  hipError_t e = hipHostMalloc((void**)&host, (size_t)roff[count] * 8, hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < count; ++i)
    e = hipMemcpyAsync(host + roff[i], rb_dev[i], nrb[i] * 8, hipMemcpyDeviceToHost, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(0);
  if (e != hipSuccess) {
    if (host) hipHostFree(host);
    release();
    return fail(PSDP_EDEVICE, std::string("set-up read-back: ") + hipGetErrorString(e));
  }
  int rc = PSDP_OK;
  std::string msg;
  for (int i = 0; i < count; ++i) {
    const int ri = setup_finish(&out[i], host + roff[i], nrb[i]);
    if (ri && !rc) {
      rc = ri;
      msg = "system " + std::to_string(i) + ": " + psdp_last_error();
    }
  }
  hipHostFree(host);
  if (rc) {
    release();
    return fail(rc, msg);
  }
  return PSDP_OK;
}

int psdp_query(const psdp_sdp* s, psdp_dims* out) {
  if (!s || !out) return fail(PSDP_EINVAL, "NULL argument");
  out->n = s->n; out->l = s->l; out->da = s->da; out->dp = s->dp; out->d1 = s->d1; out->d2 = s->d2;
  out->L0 = s->L0; out->L = s->L; out->M = s->M; out->Na = s->Na; out->Nt = s->Nt;
  out->K = s->K; out->Kpad = s->Kpad;
  const int64_t nn = (int64_t)s->n * s->n;
  int64_t pairs = 0, pairs2 = 0;
  for (int m = 0; m < s->M; ++m) {
    int z = 0;
    for (int h = 0; h < s->L0; ++h) z += s->hmask[m * s->L0 + h];
    pairs += z;
    pairs2 += (int64_t)z * (z + 1) / 2;
  }
  out->device_bytes = 8 * (s->Kpad * s->Kpad + 16 * s->Kpad + 18 * (int64_t)s->nb * nn +
                           (2 * pairs + 2 * pairs2 + s->L0) * nn) + (int64_t)s->dbytes;
  return PSDP_OK;
}

int psdp_get_polya(const psdp_sdp* s, int64_t* beta, int64_t* coef, double* H, double* scale,
                   double* cdiag) {
  if (!s) return fail(PSDP_EINVAL, "NULL handle");
  const int64_t nn = (int64_t)s->n * s->n;
  if (hipSetDevice(s->device) != hipSuccess) return fail(PSDP_EDEVICE, "hipSetDevice failed");
  if (beta) PSDP_HIP(hipMemcpy(beta, s->dbeta, (size_t)s->L0 * s->L * 8, hipMemcpyDeviceToHost));
  if (coef) PSDP_HIP(hipMemcpy(coef, s->dcoef, (size_t)s->L0 * s->M * s->Na * 8, hipMemcpyDeviceToHost));
  if (H) PSDP_HIP(hipMemcpy(H, s->dH, (size_t)s->M * s->L0 * nn * 8, hipMemcpyDeviceToHost));
  if (scale) PSDP_HIP(hipMemcpy(scale, s->dscale, (size_t)s->nb * 8, hipMemcpyDeviceToHost));
  if (cdiag) PSDP_HIP(hipMemcpy(cdiag, s->dcdiag, (size_t)s->nb * 8, hipMemcpyDeviceToHost));
  return PSDP_OK;
}

int psdp_basis(const psdp_sdp* s, int* pairs) {
  if (!s || !pairs) return fail(PSDP_EINVAL, "NULL argument");
  std::memcpy(pairs, s->basis.pairs.data(), s->basis.pairs.size() * sizeof(int));
  return PSDP_OK;
}

void psdp_free(psdp_sdp* s) {
  if (!s) return;
  if (s->dmem) hipFree(s->dmem);
  delete s;
}

int psdp_ipm_solve(psdp_sdp* sdp, const psdp_opts* opts, psdp_result* res) {
  if (!sdp || !res) return fail(PSDP_EINVAL, "NULL argument");
  return solve_batch(&sdp, 1, opts, res);
}

int psdp_ipm_solve_batched(psdp_sdp* const* sdps, int count, const psdp_opts* opts,
                           psdp_result* res) {
  if (!sdps || !res || count < 1) return fail(PSDP_EINVAL, "bad batch arguments");
  for (int i = 0; i < count; ++i)
    if (!sdps[i]) return fail(PSDP_EINVAL, "NULL handle in batch");
  return solve_batch(sdps, count, opts, res);
}

int psdp_eval_newton(psdp_sdp* sdp, const double* X, const double* Z, const double* y,
                     double* Zi, double* BTy, double* BX, double* Lam, double* LamL, double* sol,
                     void* stream) {
  if (!sdp || !X || !Z || !y) return fail(PSDP_EINVAL, "NULL argument");
  return eval_newton(sdp, X, Z, y, Zi, BTy, BX, Lam, LamL, sol, (hipStream_t)stream);
}

int psdp_eval_ladder(psdp_sdp* sdp, const double* V, const double* dV, const psdp_opts* opts,
                     double* step, int* kstar) {
  if (!sdp || !V || !dV || !step || !kstar) return fail(PSDP_EINVAL, "NULL argument");
  return eval_ladder(sdp, V, dV, opts, step, kstar);
}

}  // extern "C"
