// Homogeneous representation of A on a (translated) simplex and the
// robust-stability bisection of Section V (Examples 1 and 2).
//
// Section II makes a non-homogeneous A(alpha) homogeneous by multiplying each
// monomial of degree k by (sum alpha)^(da - k).  Section V's examples certify
// stability on simplices translated away from the unit one: the parameter x
// ranges over the image of Delta_l under a linear map x = G alpha, so
// A(G alpha) is again a polynomial in alpha.  Both steps are small host-side
// polynomial expansions (matrix coefficients times scalar polynomials of a
// few variables); every SDP they produce is set up and solved by the device
// path.  The bisection moves a parameter t of G(t) = G0 + t G1 and solves
// several trial values of t per round as one batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace psdp {
namespace {

// a homogeneous scalar polynomial in l variables: exponent -> coefficient
using Poly = std::map<std::vector<int>, double>;

Poly mul_linear(const Poly& p, const double* g, int l) {
  Poly out;
  for (const auto& kv : p)
    for (int j = 0; j < l; ++j) {
      if (g[j] == 0.0) continue;
      std::vector<int> e = kv.first;
      e[j] += 1;
      out[e] += kv.second * g[j];
    }
  return out;
}

// W_d in descending lexicographic order (Notation): alpha_1^d first
void monomials(int l, int d, int pos, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (pos == l - 1) {
    cur[pos] = d;
    out.push_back(cur);
    return;
  }
  for (int v = d; v >= 0; --v) {
    cur[pos] = v;
    monomials(l, d - v, pos + 1, cur, out);
  }
}

}  // namespace
}  // namespace psdp

using namespace psdp;

int psdp_poly_on_simplex(int n, int lx, int count, const int* exps, const double* mats, int l,
                         const double* G, int da, double* out) {
  if (n < 1 || lx < 1 || l < 1 || count < 1 || da < 0 || !exps || !mats || !out)
    return fail(PSDP_EINVAL, "psdp_poly_on_simplex: bad arguments");
  if (!G && lx != l) return fail(PSDP_EINVAL, "psdp_poly_on_simplex: G = NULL needs lx = l");
  if (da > kMaxDeg) return fail(PSDP_EOVERFLOW, "psdp_poly_on_simplex: degree above 20");
  const int64_t nn = (int64_t)n * n;
  for (int64_t i = 0; i < (int64_t)count * nn; ++i)
    if (!std::isfinite(mats[i])) return fail(PSDP_EINVAL, "psdp_poly_on_simplex: non-finite coefficient");
  if (G)
    for (int64_t i = 0; i < (int64_t)lx * l; ++i)
      if (!std::isfinite(G[i])) return fail(PSDP_EINVAL, "psdp_poly_on_simplex: non-finite map");
  std::vector<std::vector<int>> W;
  std::vector<int> cur(l, 0);
  monomials(l, da, 0, cur, W);
  std::map<std::vector<int>, int> idx;
  for (size_t i = 0; i < W.size(); ++i) idx[W[i]] = (int)i;
  std::memset(out, 0, W.size() * nn * sizeof(double));
  std::vector<double> ident(l), ones(l, 1.0);
  for (int t = 0; t < count; ++t) {
    const int* lam = exps + (int64_t)t * lx;
    int k = 0;
    for (int i = 0; i < lx; ++i) {
      if (lam[i] < 0) return fail(PSDP_EINVAL, "psdp_poly_on_simplex: negative exponent");
      k += lam[i];
    }
    if (k > da) return fail(PSDP_EINVAL, "psdp_poly_on_simplex: a term's degree exceeds da");
    // (G alpha)^lam, then times (sum alpha)^(da - k)
    Poly p;
    p[std::vector<int>(l, 0)] = 1.0;
    for (int i = 0; i < lx; ++i)
      for (int e = 0; e < lam[i]; ++e) {
        const double* g = G ? G + (int64_t)i * l : nullptr;
        if (!g) {
          for (int j = 0; j < l; ++j) ident[j] = j == i ? 1.0 : 0.0;
          g = ident.data();
        }
        p = mul_linear(p, g, l);
      }
    for (int e = k; e < da; ++e) p = mul_linear(p, ones.data(), l);
    const double* M = mats + (int64_t)t * nn;
    for (const auto& kv : p) {
      double* o = out + (int64_t)idx.at(kv.first) * nn;
      for (int64_t q = 0; q < nn; ++q) o[q] += kv.second * M[q];
    }
  }
  return PSDP_OK;
}

int psdp_bisect_simplex(int n, int lx, int count, const int* exps, const double* mats, int l,
                        const double* G0, const double* G1, int dp, int d, double t_feas,
                        double t_infeas, double tol, int width, const psdp_setup_opts* so,
                        const psdp_opts* opts, double* t_cert, double* t_other, psdp_bisect_rec* recs,
                        int rec_cap, int* nrec) {
  if (!G0 || !G1 || !t_cert || !t_other || width < 1 || width > 64 || !(tol > 0.0) ||
      !std::isfinite(t_feas) || !std::isfinite(t_infeas) || (rec_cap > 0 && !recs))
    return fail(PSDP_EINVAL, "psdp_bisect_simplex: bad arguments");
  int da = 0;
  for (int t = 0; t < count; ++t) {
    int k = 0;
    for (int i = 0; i < lx; ++i) k += exps ? exps[(int64_t)t * lx + i] : 0;
    da = std::max(da, k);
  }
  psdp_setup_opts sopt;
  psdp_setup_opts_default(&sopt);
  if (so) sopt = *so;
  sopt.da = da;
  sopt.a_on_device = 0;
  int64_t Na = 1;
  for (int i = 1; i < l; ++i) Na = Na * (da + i) / i;   // card W_da
  const int64_t nn = (int64_t)n * n;
  std::vector<double> Ab((size_t)width * Na * nn), Gt((size_t)lx * l);
  int nr = 0;
  if (nrec) *nrec = 0;
  *t_cert = NAN;
  *t_other = t_infeas;
  // solves the trial values ts (one batch); verdicts out
  auto trials = [&](const std::vector<double>& ts, std::vector<int>& ver) -> int {
    const int w = (int)ts.size();
    std::vector<const double*> aptr(w);
    for (int i = 0; i < w; ++i) {
      for (int64_t q = 0; q < (int64_t)lx * l; ++q) Gt[q] = G0[q] + ts[i] * G1[q];
      double* Ai = Ab.data() + (size_t)i * Na * nn;
      if (int rc = psdp_poly_on_simplex(n, lx, count, exps, mats, l, Gt.data(), da, Ai)) return rc;
      aptr[i] = Ai;
    }
    std::vector<int> nv(w, n), lv(w, l), dpv(w, dp), dv(w, d);
    std::vector<psdp_sdp*> h(w, nullptr);
    if (int rc = psdp_polya_setup_batched(w, aptr.data(), nv.data(), lv.data(), dpv.data(), dv.data(), &sopt,
                                          h.data()))
      return rc;
    std::vector<psdp_result> res(w);
    std::memset(res.data(), 0, w * sizeof(psdp_result));
    const int rc = psdp_ipm_solve_batched(h.data(), w, opts, res.data());
    for (auto* p : h) psdp_free(p);
    if (rc) return rc;
    ver.assign(w, PSDP_UNKNOWN);
    for (int i = 0; i < w; ++i) {
      ver[i] = res[i].verdict;
      if (nr < rec_cap)
        recs[nr] = psdp_bisect_rec{ts[i], res[i].verdict, res[i].iterations + res[i].phase1_iterations,
                                   res[i].margin};
      ++nr;
    }
    if (nrec) *nrec = std::min(nr, rec_cap);
    return PSDP_OK;
  };
  std::vector<int> ver;
  if (int rc = trials({t_feas}, ver)) return rc;
  if (ver[0] != PSDP_FEASIBLE) return PSDP_OK;
  double a = t_feas, b = t_infeas;
  while (std::fabs(a - b) > tol) {
    // width points splitting [a, b] evenly; the certified ones form the new
    // feasible end up to the first point without a certificate
    std::vector<double> ts(width);
    for (int i = 0; i < width; ++i) ts[i] = a + (b - a) * (i + 1) / (width + 1);
    if (int rc = trials(ts, ver)) return rc;
    double na = a, nb = b;
    for (int i = 0; i < width; ++i) {
      if (ver[i] == PSDP_FEASIBLE) {
        na = ts[i];
      } else {
        nb = ts[i];
        break;
      }
    }
    a = na;
    b = nb;
  }
  *t_cert = a;
  *t_other = b;
  return PSDP_OK;
}
