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
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
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

// What the set-up kernels need of one system; one array of these serves a
// whole set-up call, and each kernel's grid is the concatenation of the
// systems' grids (prefix table pre[count + 1] of their block counts).
struct SetupDesc {
  const int* Wp;
  const int* WL;
  const int* WM;
  const int* Wa;
  const double* Asrc;   // device vertices to gather into A, or null (uploaded)
  double* A;
  int64_t* beta;
  double* betaf;
  int64_t* coef;
  double* H;
  double* Hh;           // discrete form: the 2n x 2n [[-b/2 I, -H], [0, -b/2 I]]; else null
  double* scale;
  double* cdiag;
  double* bad;
  double delta, eps;
  int64_t nA;           // Na n^2
  int l, L0, L, M, Na, n, d1, d2, dp, dM, da;
};

constexpr int kGatherBlock = 1024;   // doubles per workgroup of the vertex gather

// the system whose block range holds block b (largest i with pre[i] <= b)
__device__ inline int find_sys(const int64_t* __restrict__ pre, int count, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// d! / prod delta_i! by successive exact divisions (each partial quotient is
// an integer because the remaining denominators divide the remaining
// numerator).
__device__ inline int64_t dev_multinomial(int d, const int* delta, int l) {
  int64_t r = c_fact[d];
  for (int i = 0; i < l; ++i) r /= c_fact[delta[i]];
  return r;
}

// device-resident vertices into the handle's own copy
__global__ void k_gather_A(const SetupDesc* __restrict__ D, const int64_t* __restrict__ pre,
                           int count) {
  const int i = find_sys(pre, count, blockIdx.x);
  const SetupDesc& s = D[i];
  const int64_t e0 = ((int64_t)blockIdx.x - pre[i]) * kGatherBlock;
  for (int k = threadIdx.x; k < kGatherBlock; k += blockDim.x) {
    const int64_t e = e0 + k;
    if (e < s.nA) s.A[e] = s.Asrc[e];
  }
}

// beta_{h,j} = d1! / (w_j - w_h)! for w_j >= w_h, else 0 (one thread each)
__global__ void k_beta(const SetupDesc* __restrict__ D, const int64_t* __restrict__ pre,
                       int count) {
  const int i = find_sys(pre, count, blockIdx.x);
  const SetupDesc& s = D[i];
  const int64_t t = ((int64_t)blockIdx.x - pre[i]) * blockDim.x + threadIdx.x;
  if (t >= (int64_t)s.L0 * s.L) return;
  const int h = (int)(t / s.L), j = (int)(t % s.L);
  const int l = s.l;
  int delta[32];
  bool ok = true;
  for (int q = 0; q < l; ++q) {
    delta[q] = s.WL[j * l + q] - s.Wp[h * l + q];
    ok = ok && delta[q] >= 0;
  }
  const int64_t v = ok ? dev_multinomial(s.d1, delta, l) : 0;
  s.beta[t] = v;
  s.betaf[t] = (double)v;
}

// one workgroup per (m, h): integer weights c[h][m][lam] into LDS, then
// H[m][h] = sum_lam c * A_lam entrywise.
__global__ void k_coef_H(const SetupDesc* __restrict__ D, const int64_t* __restrict__ pre,
                         int count) {
  extern __shared__ int64_t s_c[];
  const int i = find_sys(pre, count, blockIdx.x);
  const SetupDesc& s = D[i];
  const int64_t loc = (int64_t)blockIdx.x - pre[i];
  const int m = (int)(loc / s.L0), h = (int)(loc % s.L0);
  const int l = s.l, Na = s.Na, M = s.M;
  for (int lam = threadIdx.x; lam < Na; lam += blockDim.x) {
    int delta[32];
    bool ok = true;
    for (int q = 0; q < l; ++q) {
      delta[q] = s.WM[m * l + q] - s.Wp[h * l + q] - s.Wa[lam * l + q];
      ok = ok && delta[q] >= 0;
    }
    const int64_t v = ok ? dev_multinomial(s.d2, delta, l) : 0;
    s_c[lam] = v;
    s.coef[((int64_t)h * M + m) * Na + lam] = v;
  }
  __syncthreads();
  const int nn = s.n * s.n;
  const double* A = s.A;
  double* out = s.H + ((int64_t)m * s.L0 + h) * nn;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    double acc = 0.0;
    for (int lam = 0; lam < Na; ++lam) {
      const int64_t c = s_c[lam];
      if (c != 0) acc = acc + (double)c * A[(int64_t)lam * nn + e];
    }
    out[e] = acc;
  }
}

// Discrete form, one workgroup per (m, h) after k_coef_H:
// Hh[m][h] = [[-b/2 I, -H[m][h]], [0, -b/2 I]] with b = (da+d2)!/(gamma_m-h)!
// (0 unless gamma_m >= h): the coefficient of alpha^gamma_m in
// alpha^h (sum alpha)^(da+d2), which multiplies P_h on the diagonal of the
// 2n x 2n Polya coefficient [[b P, P H], [H^T P, b P]] = -(Hh^T Eh + Eh Hh).
__global__ void k_hat_H(const SetupDesc* __restrict__ D, const int64_t* __restrict__ pre, int count) {
  const int i = find_sys(pre, count, blockIdx.x);
  const SetupDesc& s = D[i];
  if (!s.Hh) return;
  const int64_t loc = (int64_t)blockIdx.x - pre[i];
  const int m = (int)(loc / s.L0), h = (int)(loc % s.L0);
  const int l = s.l, n = s.n, n2 = 2 * s.n;
  int delta[32];
  bool ok = true;
  for (int q = 0; q < l; ++q) {
    delta[q] = s.WM[m * l + q] - s.Wp[h * l + q];
    ok = ok && delta[q] >= 0;
  }
  const double hb = ok ? -0.5 * (double)dev_multinomial(s.da + s.d2, delta, l) : 0.0;
  const double* Hs = s.H + ((int64_t)m * s.L0 + h) * n * n;
  double* out = s.Hh + ((int64_t)m * s.L0 + h) * n2 * n2;
  for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
    const int r = e / n2, c = e % n2;
    double v = 0.0;
    if (r == c) v = hb;
    else if (r < n && c >= n) v = -Hs[r * n + (c - n)];
    out[e] = v;
  }
}

// *bad = 1 if any entry of the system's A is not finite (one workgroup per
// system)
__global__ void k_nonfinite(const SetupDesc* __restrict__ D) {
  const SetupDesc& s = D[blockIdx.x];
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t e = threadIdx.x; e < s.nA; e += blockDim.x) mine |= !isfinite(s.A[e]);
  if (mine) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) *s.bad = any ? 1.0 : 0.0;
}

__global__ void k_scale(const SetupDesc* __restrict__ D, const int64_t* __restrict__ pre,
                        int count) {
  const int i = find_sys(pre, count, blockIdx.x);
  const SetupDesc& s = D[i];
  const int j = (int)(((int64_t)blockIdx.x - pre[i]) * blockDim.x + threadIdx.x);
  const int L = s.L, l = s.l;
  if (j >= L + s.M) return;
  if (j < L) {
    // eq. Cj: s_j = sum_h beta_{h,j} dp!/h!
    int64_t v = 0;
    for (int h = 0; h < s.L0; ++h) v += s.beta[h * L + j] * dev_multinomial(s.dp, s.Wp + h * l, l);
    s.scale[j] = (double)v;
    s.cdiag[j] = s.delta * (double)v;
  } else {
    const int64_t v = dev_multinomial(s.dM, s.WM + (j - L) * l, l);
    s.scale[j] = (double)v;
    s.cdiag[j] = s.eps * (double)v;
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
  o->form = PSDP_FORM_CONTINUOUS;
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
  o->chol_shift_max = 1e-6;
  o->chol_shift_force = 0.0;
  o->stop_rule = PSDP_STOP_RELATIVE;
  o->sigma_rule = PSDP_SIGMA_FIXED;
  o->chol_panels = 0;
  o->chol_subpanels = 0;
}

const char* psdp_last_error(void) { return g_err.c_str(); }

const char* psdp_version(void) { return "polyaipm 0.1 (gfx950)"; }

// Host part of one system's set-up: checks, dimensions, exponent tables,
// masks and the tiled basis.  Allocates no device memory.
static int plan_system(const double* A, int n, int l, int dp, int d, const psdp_setup_opts& opt,
                       psdp_sdp** out) {
  if (!A) return fail(PSDP_EINVAL, "A is NULL");
  const int da = opt.da;
  const int d1 = opt.d1 >= 0 ? opt.d1 : d;
  const int d2 = opt.d2 >= 0 ? opt.d2 : d;
  if (n < 1 || n > kMaxN) return fail(PSDP_EINVAL, "n must be in [1, 128]");
  if (l < 1 || l > 32) return fail(PSDP_EINVAL, "l must be in [1, 32]");
  if (dp < 0 || da < 1 || d1 < 0 || d2 < 0) return fail(PSDP_EINVAL, "negative degree");
  if (opt.form != PSDP_FORM_CONTINUOUS && opt.form != PSDP_FORM_DISCRETE)
    return fail(PSDP_EINVAL, "invalid form");
  if (opt.form == PSDP_FORM_DISCRETE && n > kMaxN / 2)
    return fail(PSDP_EINVAL, "the discrete form takes n in [1, 64] (blocks of order 2n)");
  if (!(opt.delta > 0.0) || !(opt.eps >= 0.0) || !std::isfinite(opt.delta) ||
      !std::isfinite(opt.eps))
    return fail(PSDP_EINVAL, "delta must be > 0 and eps >= 0");
  if (dp + d1 > kMaxDeg || dp + da + d2 > kMaxDeg)
    return fail(PSDP_EOVERFLOW, "Polya degree above 20: multinomials exceed int64");
  const int64_t L0 = binom(l + dp - 1, l - 1), L = binom(l + dp + d1 - 1, l - 1);
  const int64_t M = binom(l + dp + da + d2 - 1, l - 1), Na = binom(l + da - 1, l - 1);
  const int64_t Nt = (int64_t)n * (n + 1) / 2;
  const int64_t K = L0 * Nt;
  if (L0 > 100000 || L > 10000000 || M > 10000000 || Na > 4096 || K > 200000 ||
      L0 * L > INT32_MAX || L0 * M > INT32_MAX)
    return fail(PSDP_EOVERFLOW, "problem dimensions too large");
  if (!opt.a_on_device) {
    for (int64_t i = 0; i < Na * n * n; ++i)
      if (!std::isfinite(A[i])) return fail(PSDP_EINVAL, "A has a non-finite entry");
  }
  psdp_sdp* s = new psdp_sdp();
  s->n = n; s->l = l; s->da = da; s->dp = dp; s->d1 = d1; s->d2 = d2;
  s->form = opt.form;
  s->bo = opt.form == PSDP_FORM_DISCRETE ? 2 * n : n;
  s->L0 = (int)L0; s->L = (int)L; s->M = (int)M; s->Na = (int)Na; s->Nt = (int)Nt;
  s->nb = (int)(L + M);
  s->K = K;
  s->Kpad = round_up(K, kNB);
  s->delta = opt.delta;
  s->eps = opt.paper_literal ? 0.0 : opt.eps;
  s->paper_literal = opt.paper_literal;
  s->device = -1;
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
  *out = s;
  return PSDP_OK;
}

// The factorial table goes to constant memory once per device.
static int upload_factorials(int dev) {
  static std::mutex mu;
  static bool done[64] = {false};
  if (dev < 0 || dev >= 64) return fail(PSDP_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> g(mu);
  if (done[dev]) return PSDP_OK;
  int64_t fact[kMaxDeg + 1];
  for (int i = 0; i <= kMaxDeg; ++i) fact[i] = host_fact(i);
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_fact), fact, sizeof(fact)) != hipSuccess)
    return fail(PSDP_EDEVICE, "copy of the factorial table failed");
  done[dev] = true;
  return PSDP_OK;
}

// Set-up of count systems with one device block shared by their handles:
// one upload (descriptors, block prefix tables, exponent tables and host
// vertices), one launch per set-up kernel over all systems, one read-back
// (betaf, scale, cdiag and the non-finite flag of A of every system, held
// contiguously).  label: prefix error messages with the failing system.
static int setup_many(int count, const double* const* A, const int* n, const int* l,
                      const int* dp, const int* d, const psdp_setup_opts* o, psdp_sdp** out,
                      bool label) {
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  auto release = [&]() {
    for (int i = 0; i < count; ++i) {
      delete out[i];
      out[i] = nullptr;
    }
  };
  auto fail_sys = [&](int i, int code, const std::string& msg) {
    release();
    return fail(code, label ? "system " + std::to_string(i) + ": " + msg : msg);
  };
  try {
    psdp_setup_opts opt;
    psdp_setup_opts_default(&opt);
    if (o) opt = *o;
    for (int i = 0; i < count; ++i) {
      const int rc = plan_system(A[i], n[i], l[i], dp[i], d[i], opt, &out[i]);
      if (rc) return fail_sys(i, rc, psdp_last_error());
    }
    if (count == 0) return PSDP_OK;
    // first device call: after every argument has been checked
    int dev = 0;
    if (const hipError_t e = hipGetDevice(&dev)) {
      release();
      return fail(PSDP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < count; ++i) out[i]->device = dev;
    if (const int rc = upload_factorials(dev)) {
      const std::string msg = psdp_last_error();
      release();
      return fail(rc, msg);
    }

    // layout of the block: [upload | read-back | work]
    const bool dev_a = opt.a_on_device != 0;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    std::vector<int64_t> preA(count + 1, 0), preB(count + 1, 0), preH(count + 1, 0),
        preS(count + 1, 0), roff(count + 1, 0);
    std::vector<size_t> oTab(count), oAu(count), oWork(count);
    size_t up = al(count * sizeof(SetupDesc)) + 4 * al((count + 1) * sizeof(int64_t));
    const size_t oPre = al(count * sizeof(SetupDesc));
    int maxNa = 1;
    for (int i = 0; i < count; ++i) {
      const psdp_sdp* s = out[i];
      const int64_t nA = (int64_t)s->Na * s->n * s->n;
      const size_t ntab = s->basis.pairs.size() + s->Wp.size() + s->WL.size() + s->WM.size() +
                          s->Wa.size();
      oTab[i] = up;
      up += al(ntab * 4);
      oAu[i] = up;
      if (!dev_a) up += al(nA * 8);
      preA[i + 1] = preA[i] + (dev_a ? (nA + kGatherBlock - 1) / kGatherBlock : 0);
      preB[i + 1] = preB[i] + ((int64_t)s->L0 * s->L + 255) / 256;
      preH[i + 1] = preH[i] + (int64_t)s->M * s->L0;
      preS[i + 1] = preS[i] + ((int64_t)s->L + s->M + 255) / 256;
      roff[i + 1] = roff[i] + (int64_t)s->L0 * s->L + 2 * ((int64_t)s->L + s->M) + 1;
      maxNa = std::max(maxNa, s->Na);
    }
    if (preB[count] > INT32_MAX || preH[count] > INT32_MAX || preS[count] > INT32_MAX ||
        preA[count] > INT32_MAX) {
      release();
      return fail(PSDP_EOVERFLOW, "set-up grids too large for one call");
    }
    const size_t oRb = al(up);
    size_t off = oRb + al(roff[count] * 8);
    for (int i = 0; i < count; ++i) {
      const psdp_sdp* s = out[i];
      const int64_t nA = (int64_t)s->Na * s->n * s->n;
      oWork[i] = off;
      off += al((int64_t)s->L0 * s->L * 8) + al((int64_t)s->L0 * s->M * s->Na * 8) +
             al((int64_t)s->M * s->L0 * s->n * s->n * 8) + (dev_a ? al(nA * 8) : 0) +
             (s->form == PSDP_FORM_DISCRETE ? al((int64_t)s->M * s->L0 * s->bo * s->bo * 8) : 0);
    }
    void* raw = nullptr;
    if (hipMalloc(&raw, off) != hipSuccess) {
      (void)hipGetLastError();
      release();
      return fail(PSDP_ENOMEM, "device allocation for the set-up failed");
    }
    std::shared_ptr<void> block(raw, [](void* p) { (void)hipFree(p); });
    char* base = (char*)raw;

    // host image of the upload region
    std::vector<char> img(up);
    SetupDesc* hd = (SetupDesc*)img.data();
    for (int i = 0; i < count; ++i) {
      psdp_sdp* s = out[i];
      const int64_t nA = (int64_t)s->Na * s->n * s->n;
      int* tab = (int*)(img.data() + oTab[i]);
      size_t t = 0;
      auto put = [&](const std::vector<int>& v) {
        const size_t r = t;
        std::memcpy(tab + t, v.data(), v.size() * 4);
        t += v.size();
        return r;
      };
      const size_t iBa = put(s->basis.pairs), iWp = put(s->Wp), iWL = put(s->WL),
                   iWM = put(s->WM), iWa = put(s->Wa);
      int* dtab = (int*)(base + oTab[i]);
      char* w = base + oWork[i];
      s->dbeta = (int64_t*)w;
      w += al((int64_t)s->L0 * s->L * 8);
      s->dcoef = (int64_t*)w;
      w += al((int64_t)s->L0 * s->M * s->Na * 8);
      s->dH = (double*)w;
      w += al((int64_t)s->M * s->L0 * s->n * s->n * 8);
      s->dHh = s->dH;
      if (s->form == PSDP_FORM_DISCRETE) {
        s->dHh = (double*)w;
        w += al((int64_t)s->M * s->L0 * s->bo * s->bo * 8);
      }
      if (dev_a) {
        s->dA = (double*)w;
      } else {
        s->dA = (double*)(base + oAu[i]);
        std::memcpy(img.data() + oAu[i], A[i], nA * 8);
      }
      double* rb = (double*)(base + oRb) + roff[i];
      const int64_t LL = (int64_t)s->L0 * s->L, nbk = (int64_t)s->L + s->M;
      s->dbetaf = rb;
      s->dscale = rb + LL;
      s->dcdiag = rb + LL + nbk;
      s->dbasis = dtab + iBa;
      s->dmem = block;
      s->dbytes = (oAu[i] - oTab[i]) + (dev_a ? 0 : al(nA * 8)) + (roff[i + 1] - roff[i]) * 8 +
                  (i + 1 < count ? oWork[i + 1] : off) - oWork[i];
      SetupDesc& q = hd[i];
      q.Wp = dtab + iWp;
      q.WL = dtab + iWL;
      q.WM = dtab + iWM;
      q.Wa = dtab + iWa;
      q.Asrc = dev_a ? A[i] : nullptr;
      q.A = s->dA;
      q.beta = s->dbeta;
      q.betaf = s->dbetaf;
      q.coef = s->dcoef;
      q.H = s->dH;
      q.Hh = s->form == PSDP_FORM_DISCRETE ? s->dHh : nullptr;
      q.scale = s->dscale;
      q.cdiag = s->dcdiag;
      q.bad = rb + LL + 2 * nbk;
      q.delta = s->delta;
      q.eps = s->eps;
      q.nA = nA;
      q.l = s->l; q.L0 = s->L0; q.L = s->L; q.M = s->M; q.Na = s->Na; q.n = s->n;
      q.d1 = s->d1; q.d2 = s->d2; q.dp = s->dp; q.dM = s->dp + s->da + s->d2; q.da = s->da;
    }
    const size_t pstride = al((count + 1) * sizeof(int64_t));
    const std::vector<int64_t>* pres[4] = {&preA, &preB, &preH, &preS};
    for (int k = 0; k < 4; ++k)
      std::memcpy(img.data() + oPre + k * pstride, pres[k]->data(), (count + 1) * 8);
    const SetupDesc* dD = (const SetupDesc*)base;
    const int64_t* dpre[4];
    for (int k = 0; k < 4; ++k) dpre[k] = (const int64_t*)(base + oPre + k * pstride);

    hipError_t e = hipMemcpyAsync(base, img.data(), up, hipMemcpyHostToDevice, 0);
    if (e == hipSuccess) {
      if (preA[count] > 0)
        hipLaunchKernelGGL(k_gather_A, dim3((unsigned)preA[count]), dim3(256), 0, 0, dD, dpre[0],
                           count);
      hipLaunchKernelGGL(k_beta, dim3((unsigned)preB[count]), dim3(256), 0, 0, dD, dpre[1], count);
      hipLaunchKernelGGL(k_coef_H, dim3((unsigned)preH[count]), dim3(256), maxNa * 8, 0, dD,
                         dpre[2], count);
      hipLaunchKernelGGL(k_scale, dim3((unsigned)preS[count]), dim3(256), 0, 0, dD, dpre[3], count);
      bool anyd = false;
      for (int i = 0; i < count; ++i) anyd = anyd || out[i]->form == PSDP_FORM_DISCRETE;
      if (anyd)   // after k_coef_H on the same stream
        hipLaunchKernelGGL(k_hat_H, dim3((unsigned)preH[count]), dim3(256), 0, 0, dD, dpre[2], count);
      hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)count), dim3(256), 0, 0, dD);
      e = hipGetLastError();
    }
    // one read-back (it also waits for the kernels)
    std::vector<double> rbh(roff[count]);
    if (e == hipSuccess)
      e = hipMemcpy(rbh.data(), base + oRb, roff[count] * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(0);
      release();
      return fail(PSDP_EDEVICE, std::string("set-up on the device: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < count; ++i) {
      psdp_sdp* s = out[i];
      const double* rb = rbh.data() + roff[i];
      const int64_t LL = (int64_t)s->L0 * s->L, nbk = (int64_t)s->L + s->M;
      if (rb[LL + 2 * nbk] != 0.0) return fail_sys(i, PSDP_EINVAL, "A has a non-finite entry");
      s->betaf.assign(rb, rb + LL);
      s->scale_h.assign(rb + LL, rb + LL + nbk);
      s->cdiag_h.assign(rb + LL + nbk, rb + LL + 2 * nbk);
    }
    return PSDP_OK;
  } catch (const std::bad_alloc&) {
    release();
    return fail(PSDP_ENOMEM, "host allocation failed");
  } catch (...) {
    release();
    return fail(PSDP_EINVAL, "unexpected exception in the set-up");
  }
}

int psdp_polya_setup(const double* A, int n, int l, int dp, int d, const psdp_setup_opts* o,
                     psdp_sdp** out) {
  if (!out) return fail(PSDP_EINVAL, "out is NULL");
  return setup_many(1, &A, &n, &l, &dp, &d, o, out, false);
}

int psdp_polya_setup_batched(int count, const double* const* A, const int* n, const int* l,
                             const int* dp, const int* d, const psdp_setup_opts* o, psdp_sdp** out) {
  if (count < 0) return fail(PSDP_EINVAL, "count is negative");
  if (count > 0 && (!A || !n || !l || !dp || !d || !out)) return fail(PSDP_EINVAL, "NULL argument");
  return setup_many(count, A, n, l, dp, d, o, out, true);
}

int psdp_query(const psdp_sdp* s, psdp_dims* out) {
  if (!s || !out) return fail(PSDP_EINVAL, "NULL argument");
  out->n = s->n; out->l = s->l; out->da = s->da; out->dp = s->dp; out->d1 = s->d1; out->d2 = s->d2;
  out->L0 = s->L0; out->L = s->L; out->M = s->M; out->Na = s->Na; out->Nt = s->Nt;
  out->K = s->K; out->Kpad = s->Kpad;
  out->form = s->form; out->bo = s->bo;
  const int64_t nn = (int64_t)s->bo * s->bo;
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
  // the device block goes with the last handle of its set-up call
  delete s;
}

int psdp_ipm_solve(psdp_sdp* sdp, const psdp_opts* opts, psdp_result* res) {
  if (!sdp || !res) return fail(PSDP_EINVAL, "NULL argument");
  return solve_batch(&sdp, 1, opts, res);
}

int psdp_ipm_solve_noalloc(psdp_sdp* sdp, const psdp_opts* opts, psdp_result* res) {
  if (!sdp || !res) return fail(PSDP_EINVAL, "NULL argument");
  return solve_batch(&sdp, 1, opts, res, true);
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
                     int chol_panels, int chol_subpanels, void* stream) {
  if (!sdp || !X || !Z || !y) return fail(PSDP_EINVAL, "NULL argument");
  if (chol_panels < -3 || chol_panels > 32) return fail(PSDP_EINVAL, "chol_panels must lie in [-3, 32]");
  if (chol_subpanels < 0 || (chol_subpanels > 0 && (chol_panels <= 0 || chol_panels % chol_subpanels)))
    return fail(PSDP_EINVAL, "chol_subpanels must divide a chol_panels width (0: none)");
  return eval_newton(sdp, X, Z, y, Zi, BTy, BX, Lam, LamL, sol, chol_panels, chol_subpanels,
                     (hipStream_t)stream);
}

int psdp_eval_schur(psdp_sdp* sdp, const double* X, const double* Z, int precision, double* Lam,
                    void* stream) {
  if (!sdp || !X || !Z || !Lam) return fail(PSDP_EINVAL, "NULL argument");
  return eval_schur(sdp, X, Z, precision, Lam, (hipStream_t)stream);
}

int psdp_eval_ladder(psdp_sdp* sdp, const double* V, const double* dV, const psdp_opts* opts,
                     double* step, int* kstar) {
  if (!sdp || !V || !dV || !step || !kstar) return fail(PSDP_EINVAL, "NULL argument");
  return eval_ladder(sdp, V, dV, opts, step, kstar);
}

}  // extern "C"
