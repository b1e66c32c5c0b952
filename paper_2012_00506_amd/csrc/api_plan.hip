// C ABI: slice_plan -- slice boundaries by exact inertia (Section 3.1,
// Approach-1 equal counts and Approach-2 equal widths; counts per slice from
// two inertias as in Section 3.2) -- and slice_plan_prev, slices from the
// previous eigenvalues of a sequence (Section 3.1 k-means, Algorithm
// alg:kmeans; bounds of Section 3.2, Algorithm alg:lower_upper).  Host
// control over batched GPU inertia: every round evaluates all open
// boundaries in one launch.
#include <math.h>

#include <algorithm>
#include <map>
#include <vector>

#include "planner.h"
#include "solve_job.h"

namespace fb {

struct InertiaRunner {
  const Band* bd;
  double* shifts_dev;
  int32_t* cnt_dev;
  void* scratch;
  int cap;
  hipStream_t st;
  int evals = 0;
  std::vector<int32_t> h;
  // n_-(s) for every shift, in one launch per chunk of cap shifts
  int run(const std::vector<double>& s, std::vector<int>& neg) {
    neg.assign(s.size(), 0);
    for (size_t c0 = 0; c0 < s.size(); c0 += cap) {
      int nc = (int)std::min<size_t>(cap, s.size() - c0);
      FB_HIP(hipMemcpyAsync(shifts_dev, s.data() + c0, sizeof(double) * nc, hipMemcpyHostToDevice, st));
      FB_TRY(launch_inertia(*bd, nc, shifts_dev, cnt_dev, scratch, st));
      h.resize(3 * (size_t)nc);
      FB_HIP(hipMemcpyAsync(h.data(), cnt_dev, sizeof(int32_t) * 3 * nc, hipMemcpyDeviceToHost, st));
      FB_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < nc; ++i) neg[c0 + i] = h[3 * i];
    }
    evals += (int)s.size();
    return 0;
  }
};

// Certify boundaries: n_-(s - d) = n_-(s + d), trying s + 2 d k for
// k = 0, 1, -1, 2, -2, ..., 32, -32.  All open boundaries advance together.
static int certify_all(InertiaRunner& ir, std::vector<double>& s, double delta,
                       std::vector<int>& neg_out) {
  const int nb = (int)s.size();
  std::vector<double> base = s;
  std::vector<int> open(nb, 1), tries(nb, 0);
  neg_out.assign(nb, 0);
  for (int round = 0; round < 65; ++round) {
    std::vector<double> q;
    std::vector<int> who;
    for (int i = 0; i < nb; ++i)
      if (open[i]) {
        int t = tries[i];
        double k = t == 0 ? 0.0 : (t % 2 ? (t + 1) / 2 : -(t / 2));
        double c = base[i] + 2.0 * delta * k;
        s[i] = c;
        q.push_back(c - delta);
        q.push_back(c + delta);
        who.push_back(i);
      }
    if (who.empty()) return 0;
    std::vector<int> neg;
    FB_TRY(ir.run(q, neg));
    for (size_t a = 0; a < who.size(); ++a) {
      int i = who[a];
      if (neg[2 * a] == neg[2 * a + 1]) {
        open[i] = 0;
        neg_out[i] = neg[2 * a];
      } else {
        ++tries[i];
      }
    }
  }
  for (int i = 0; i < nb; ++i)
    if (open[i]) return FB_ERR_CERTIFY;
  return 0;
}

}  // namespace fb

using namespace fb;

extern "C" int slice_plan(const fb_band* B, const fb_plan_opts* o, double* bounds,
                          int32_t* counts, int32_t* n_inertia, void* work, size_t* lwork,
                          void* stream) {
  if (check_band(B)) return -1;
  if (!o) return -2;
  if (o->mode != FB_PLAN_EQUAL_WIDTH && o->mode != FB_PLAN_EQUAL_COUNT &&
      o->mode != FB_PLAN_LEARNED)
    return -2;
  if (o->K < 1 || o->K > 1 << 20) return -2;
  if (!(o->cert_delta >= 0) || !(o->count_tol >= 0) || o->max_rounds < 0) return -2;
  if (o->mode == FB_PLAN_EQUAL_WIDTH && (isnan(o->lo) || isnan(o->hi) || !(o->lo < o->hi)))
    return -2;
  if (o->nev < 0) return -2;
  if (o->targets)
    for (int i = 0; i < o->K; ++i)
      if (o->targets[i] < 0) return -2;
  if (!bounds) return -3;
  if (!counts) return -4;
  if (!lwork) return -7;
  const int K = o->K;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  const int cap = 2 * (K + 1) + K;
  double* sh = ar.take<double>(cap);
  int32_t* cnt = ar.take<int32_t>(3 * (size_t)cap);
  size_t scb = inertia_scratch_bytes(bd, cap);
  void* scratch = scb ? (void*)ar.take<char>(scb) : nullptr;
  const bool learned = o->mode == FB_PLAN_LEARNED;
  float *xin = nullptr, *yout = nullptr, *hid = nullptr;
  Arena far;  // features scratch, carved after everything else
  if (learned && o->planner) {
    xin = ar.take<float>(kPlanFeatures);
    yout = ar.take<float>(kPlanOutputs);
    hid = ar.take<float>(kH1 + kH2);
    far.base = nullptr;
    std::vector<double> dummy(kPlanFeatures);
    FB_TRY(band_features_dev(bd, o->seed, far, dummy.data(), st));  // size query
    char* fbase = ar.take<char>(far.used + 256);
    far.base = fbase;
    far.cap = far.used + 256;
    far.used = 0;
  }
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  double stats[3];
  FB_TRY(band_stats_host(bd, stats, st));
  const double delta = o->cert_delta * stats[0];
  InertiaRunner ir{&bd, sh, cnt, scratch, cap, st};

  std::vector<double> edges;
  std::vector<int> neg;
  if (o->mode == FB_PLAN_EQUAL_WIDTH) {
    for (int i = 0; i <= K; ++i) edges.push_back(o->lo + (o->hi - o->lo) * i / K);
    edges[K] = o->hi;
    FB_TRY(certify_all(ir, edges, delta, neg));
  } else {
    // no interval: the whole spectrum, i.e. the Gershgorin interval widened
    // so that a bound that is itself an eigenvalue stays inside [lo, hi)
    const double pad = 4.0 * delta + 1e-12 * stats[0];
    double lo = isnan(o->lo) ? stats[1] - pad : o->lo;
    double hi = isnan(o->hi) ? stats[2] + pad : o->hi;
    if (!(lo < hi)) return -2;
    std::vector<double> ends = {lo, hi};
    std::vector<int> ne;
    FB_TRY(certify_all(ir, ends, delta, ne));
    lo = ends[0];
    hi = ends[1];
    int n_lo = ne[0], n_hi = ne[1];
    std::map<double, int> known = {{lo, n_lo}, {hi, n_hi}};
    // an exact total: the lowest nev eigenvalues above lo (or the sum of the
    // given slice counts) -- the upper end is bisected to the exact count
    // and certified there
    int64_t want = o->nev;
    if (want <= 0 && o->targets) {
      want = 0;
      for (int i = 0; i < K; ++i) want += o->targets[i];
    }
    if (want > 0) {
      if (want > n_hi - n_lo) return -2;
      const int tcount = n_lo + (int)want;
      double a = lo, b = hi;  // n_-(a) <= tcount < ... n_-(b) >= tcount
      int na = n_lo, nb_ = n_hi;
      bool done = false;
      // One launch evaluates the next `depth` levels of the bisection below
      // [a, b] (its 2^depth - 1 midpoints, formed as the bisection forms
      // them), so that the sequential bisection then walks them without a
      // launch per point; only the points it visits enter `known`, and the
      // plan is the one a launch per point gives.
      int depth = 1;
      while (depth < 6 && (2 << depth) - 1 <= cap) ++depth;
      std::map<double, int> spec;
      auto count_at = [&](double c, int& v) -> int {
        auto it = spec.find(c);
        if (it == spec.end()) {
          std::vector<double> tree;
          std::vector<std::pair<double, double>> lvl = {{a, b}}, nxt;
          for (int d = 0; d < depth; ++d) {
            nxt.clear();
            for (auto& ab2 : lvl) {
              const double m = 0.5 * (ab2.first + ab2.second);
              tree.push_back(m);
              nxt.push_back({ab2.first, m});
              nxt.push_back({m, ab2.second});
            }
            lvl.swap(nxt);
          }
          std::vector<int> tv;
          FB_TRY(ir.run(tree, tv));
          spec.clear();
          for (size_t q = 0; q < tree.size(); ++q) spec[tree[q]] = tv[q];
          it = spec.find(c);
          if (it == spec.end()) return FB_ERR_INTERNAL;
        }
        v = it->second;
        return 0;
      };
      for (int round = 0; round < 200 && !done; ++round) {
        double c;
        if (nb_ == tcount) {
          // b already has the count: certify it
          std::vector<double> e1 = {b};
          std::vector<int> c1;
          FB_TRY(certify_all(ir, e1, delta, c1));
          if (c1[0] == tcount) {
            hi = e1[0];
            n_hi = tcount;
            done = true;
            break;
          }
          c = 0.5 * (a + b);
        } else {
          c = 0.5 * (a + b);
        }
        int ncv = 0;
        FB_TRY(count_at(c, ncv));
        known[c] = ncv;
        if (ncv > tcount) {
          b = c;
          nb_ = ncv;
        } else if (ncv < tcount) {
          a = c;
          na = ncv;
        } else {
          b = c;
          nb_ = ncv;
        }
      }
      if (!done) return FB_ERR_CERTIFY;
      // keep only known points inside [lo, hi]
      for (auto it = known.begin(); it != known.end();)
        it = it->first > hi ? known.erase(it) : std::next(it);
      known[hi] = n_hi;
    }
    const int total = n_hi - n_lo;
    std::vector<int> target(K - 1);
    if (o->targets) {
      int64_t acc = n_lo;
      for (int i = 1; i < K; ++i) {
        acc += o->targets[i - 1];
        target[i - 1] = (int)acc;
      }
    } else {
      for (int i = 1; i < K; ++i) target[i - 1] = n_lo + (int)nearbyint((double)i * total / K);  // half to even
    }
    const int tol = (int)floor(o->count_tol * total / K);
    // Predicted fraction of eigenvalues below x as a monotone piecewise-linear
    // function through (px, py): the network's 64 outputs at the centres of
    // the Gershgorin interval's 64 cells, clipped to [0, 1] and made
    // non-decreasing; without a network, the uniform density on [lo, hi].
    std::vector<double> px, py;
    if (learned) {
      px = {stats[1]};
      py = {0.0};
      if (o->planner && K > 1) {
        std::vector<double> feat(kPlanFeatures);
        FB_TRY(band_features_dev(bd, o->seed, far, feat.data(), st));
        std::vector<float> xf(feat.begin(), feat.end());
        FB_HIP(hipMemcpyAsync(xin, xf.data(), sizeof(float) * kPlanFeatures,
                              hipMemcpyHostToDevice, st));
        FB_TRY(net_forward((const float*)o->planner, 1, xin, yout, hid, hid + kH1, st));
        std::vector<float> q(kPlanOutputs);
        FB_HIP(hipMemcpyAsync(q.data(), yout, sizeof(float) * kPlanOutputs,
                              hipMemcpyDeviceToHost, st));
        FB_HIP(hipStreamSynchronize(st));
        const double glo = stats[1], ghi = stats[2];
        double run = 0.0;
        for (int k = 0; k < kPlanOutputs; ++k) {
          double v = std::min(1.0, std::max(0.0, (double)q[k]));  // NaN -> 0
          run = std::max(run, v);
          px.push_back(glo + (k + 0.5) * (ghi - glo) / kPlanOutputs);
          py.push_back(run);
        }
        px.push_back(ghi);
        py.push_back(1.0);
      } else {
        px = {lo, hi};
        py = {(double)n_lo / bd.n, (double)n_hi / bd.n};
      }
    }
    auto fhat = [&](double x) {
      if (x <= px.front()) return py.front();
      if (x >= px.back()) return py.back();
      size_t j = std::upper_bound(px.begin(), px.end(), x) - px.begin();
      double t = (x - px[j - 1]) / (px[j] - px[j - 1]);
      return py[j - 1] + t * (py[j] - py[j - 1]);
    };
    auto finv = [&](double y) {  // smallest x with fhat(x) >= y
      if (y <= py.front()) return px.front();
      if (y >= py.back()) return px.back();
      size_t j = std::lower_bound(py.begin(), py.end(), y) - py.begin();
      if (py[j] <= py[j - 1]) return px[j];
      return px[j - 1] + (px[j] - px[j - 1]) * (y - py[j - 1]) / (py[j] - py[j - 1]);
    };
    std::vector<double> found(K - 1, NAN);
    std::vector<char> have(K - 1, 0);
    // bracket widths one and two rounds ago
    std::vector<double> w1(K - 1, INFINITY), w2(K - 1, INFINITY);
    for (int round = 0; round < o->max_rounds; ++round) {
      std::vector<double> xs;
      std::vector<int> vs;
      for (auto& kv : known) {
        xs.push_back(kv.first);
        vs.push_back(kv.second);
      }
      std::vector<double> shifts;
      for (int i = 0; i < K - 1; ++i) {
        if (have[i]) continue;
        const int t = target[i];
        int ia = 0;
        for (size_t j = 0; j < xs.size(); ++j)
          if (vs[j] <= t) ia = (int)j;
        int ib = std::min<int>(ia + 1, (int)xs.size() - 1);
        if (abs(vs[ia] - t) <= tol) {
          found[i] = xs[ia];
          have[i] = 1;
        } else if (abs(vs[ib] - t) <= tol) {
          found[i] = xs[ib];
          have[i] = 1;
        } else {
          const double xa = xs[ia], xb = xs[ib], w = xb - xa;
          double s = 0.5 * (xa + xb);
          if (learned && w <= 0.5 * w2[i]) {
            // The exact counts at the bracket ends rescale the predicted
            // distribution inside it; invert it at the target.  A bracket
            // that did not halve over the last two rounds is bisected.
            // Inside two cells of the prediction the network has nothing
            // to add to the exact counts: plain linear interpolation.
            const double fa = fhat(xa), fb = fhat(xb);
            const double frac = (double)(t - vs[ia]) / (double)(vs[ib] - vs[ia]);
            const double cell = (px.back() - px.front()) / kPlanOutputs;
            double g = (fb > fa && w > 2.0 * cell) ? finv(fa + frac * (fb - fa)) : xa + frac * w;
            s = std::min(xb - 0.01 * w, std::max(xa + 0.01 * w, g));
          }
          w2[i] = w1[i];
          w1[i] = w;
          shifts.push_back(s);
        }
      }
      if (shifts.empty()) break;
      std::vector<double> fresh;
      for (double s : shifts)
        if (!known.count(s) && std::find(fresh.begin(), fresh.end(), s) == fresh.end())
          fresh.push_back(s);
      std::vector<int> fv;
      FB_TRY(ir.run(fresh, fv));
      for (size_t j = 0; j < fresh.size(); ++j) known[fresh[j]] = fv[j];
    }
    for (int i = 0; i < K - 1; ++i) {
      if (have[i]) continue;
      // round cap reached: the known point whose count is closest to the target
      double best = NAN;
      int bd_ = 0;
      for (auto& kv : known) {
        int d = abs(kv.second - target[i]);
        if (isnan(best) || d < bd_) {
          best = kv.first;
          bd_ = d;
        }
      }
      found[i] = best;
    }
    std::vector<int> inner_neg;
    FB_TRY(certify_all(ir, found, delta, inner_neg));
    edges.push_back(lo);
    neg.push_back(n_lo);
    for (int i = 0; i < K - 1; ++i) {
      edges.push_back(found[i]);
      neg.push_back(inner_neg[i]);
    }
    edges.push_back(hi);
    neg.push_back(n_hi);
  }
  for (int i = 0; i <= K; ++i) bounds[i] = edges[i];
  for (int i = 0; i < K; ++i) counts[i] = neg[i + 1] - neg[i];
  if (n_inertia) *n_inertia = ir.evals;
  return 0;
}

// ---------------------------------------------------------------- from previous eigenvalues
namespace fb {

// Simplified one-dimensional k-means of ascending d[0..n) into at most K
// groups of consecutive points, held as split indices s (s[0] = 0, s.back()
// = n); see slice_plan_prev in the header for the rule.
static void kmeans_1d(const double* d, int64_t n, int K, int max_sweeps,
                      std::vector<int64_t>& s) {
  const int64_t q = n / K, r = n % K;
  s.assign(1, 0);
  for (int i = 0; i < K; ++i) s.push_back(s.back() + (i < r ? q + 1 : q));
  s.erase(std::unique(s.begin(), s.end()), s.end());  // groups with no point
  auto cen = [&](int64_t a, int64_t b) { return 0.5 * (d[a] + d[b - 1]); };
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    const std::vector<int64_t> old = s;
    for (size_t j = 1; j + 1 < s.size(); ++j) {
      if (s[j] <= s[j - 1] || s[j + 1] <= s[j]) continue;
      const double c = 0.5 * (cen(s[j - 1], s[j]) + cen(s[j], s[j + 1]));
      s[j] = std::upper_bound(d, d + n, c) - d;
    }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    if (s == old) break;
  }
}

}  // namespace fb

extern "C" int slice_plan_prev(const fb_band* B, const double* prev, int64_t nprev,
                               const fb_prev_opts* o, double* bounds, int32_t* counts,
                               int32_t* K_out, int32_t* n_inertia, void* work, size_t* lwork,
                               void* stream) {
  if (check_band(B)) return -1;
  if (!prev || nprev < 1) return -2;
  for (int64_t i = 0; i < nprev; ++i)
    if (!isfinite(prev[i]) || (i > 0 && prev[i] < prev[i - 1])) return -2;
  if (!o || o->K < 1 || o->K > 1 << 20 || o->nev < 1 || o->nev > nprev) return -4;
  if (!(o->alpha >= 0) || o->m1 < 0 || !(o->cert_delta >= 0) || o->max_sweeps < 0 ||
      o->max_steps < 1)
    return -4;
  if (!bounds) return -5;
  if (!counts) return -6;
  if (!lwork) return -10;
  const int K = o->K;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  const int cap = 2 * (K + 1);
  double* sh = ar.take<double>(cap);
  int32_t* cnt = ar.take<int32_t>(3 * (size_t)cap);
  size_t scb = inertia_scratch_bytes(bd, cap);
  void* scratch = scb ? (void*)ar.take<char>(scb) : nullptr;
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  double stats[3];
  FB_TRY(band_stats_host(bd, stats, st));
  const double nrm = stats[0];
  const double delta = o->cert_delta * nrm;
  const double floor_ = 4.0 * o->cert_delta * nrm + 1e-12 * nrm;
  InertiaRunner ir{&bd, sh, cnt, scratch, cap, st};
  const int64_t nev = o->nev;
  auto step = [&](double a, double gap) {
    return std::max(std::max(o->alpha * fabs(a), (double)o->m1 * gap), floor_);
  };
  // lower bound: below every eigenvalue
  double b0;
  {
    const double s0 = step(prev[0], nprev >= 2 ? prev[1] - prev[0] : 0.0);
    double b = prev[0] - s0;
    bool ok = false;
    for (int it = 0; it < o->max_steps && !ok; ++it) {
      std::vector<int> v;
      FB_TRY(ir.run({b}, v));
      if (v[0] == 0)
        ok = true;
      else
        b = b - s0;
    }
    if (!ok) return FB_ERR_CERTIFY;
    b0 = b;
  }
  // upper bound: at least nev eigenvalues below
  double bK;
  {
    const double s1 = step(prev[nev - 1], nev >= 2 ? prev[nev - 1] - prev[nev - 2] : 0.0);
    double b = prev[nev - 1] + s1;
    bool ok = false;
    for (int it = 0; it < o->max_steps && !ok; ++it) {
      std::vector<int> v;
      FB_TRY(ir.run({b}, v));
      if (v[0] >= nev)
        ok = true;
      else
        b = b + s1;
    }
    if (!ok) return FB_ERR_CERTIFY;
    bK = b;
  }
  std::vector<int64_t> sp;
  kmeans_1d(prev, nev, K, o->max_sweeps, sp);
  std::vector<double> edges = {b0};
  for (size_t j = 1; j + 1 < sp.size(); ++j) edges.push_back(0.5 * (prev[sp[j] - 1] + prev[sp[j]]));
  edges.push_back(bK);
  std::vector<int> neg;
  FB_TRY(certify_all(ir, edges, delta, neg));
  const int Kp = (int)edges.size() - 1;
  for (int i = 0; i < Kp; ++i)
    if (!(edges[i + 1] > edges[i])) return FB_ERR_CERTIFY;
  for (int i = 0; i <= Kp; ++i) bounds[i] = edges[i];
  for (int i = 0; i < Kp; ++i) counts[i] = neg[i + 1] - neg[i];
  if (K_out) *K_out = Kp;
  if (n_inertia) *n_inertia = ir.evals;
  return 0;
}

extern "C" int32_t fb_m0_rule(int32_t m) {
  if (m < 0) return -1;
  const int64_t a = ((int64_t)3 * m + 1) / 2;  // ceil(1.5 m)
  const int64_t v = std::max<int64_t>(a, (int64_t)m + 10);
  return v > INT32_MAX ? INT32_MAX : (int32_t)v;
}

extern "C" int slice_certify(const fb_band* B, int32_t nb, double* bounds, double cert_delta,
                             int32_t* neg, int32_t* counts, int32_t* m0, int32_t* n_inertia,
                             void* work, size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (nb < 1 || nb > (1 << 20)) return -2;
  if (!bounds) return -3;
  for (int i = 0; i < nb; ++i)
    if (!isfinite(bounds[i]) || (i > 0 && !(bounds[i] > bounds[i - 1]))) return -3;
  if (!(cert_delta >= 0) || !isfinite(cert_delta)) return -4;
  if (!neg) return -5;
  if (nb > 1 && !counts) return -6;
  if (!lwork) return -10;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  const int cap = 2 * nb;
  double* sh = ar.take<double>(cap);
  int32_t* cnt = ar.take<int32_t>(3 * (size_t)cap);
  size_t scb = inertia_scratch_bytes(bd, cap);
  void* scratch = scb ? (void*)ar.take<char>(scb) : nullptr;
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  double stats[3];
  FB_TRY(band_stats_host(bd, stats, st));
  InertiaRunner ir{&bd, sh, cnt, scratch, cap, st};
  std::vector<double> edges(bounds, bounds + nb);
  std::vector<int> ng;
  FB_TRY(certify_all(ir, edges, cert_delta * stats[0], ng));
  for (int i = 0; i + 1 < nb; ++i)
    if (!(edges[i + 1] > edges[i])) return FB_ERR_CERTIFY;  // two boundaries met
  for (int i = 0; i < nb; ++i) {
    bounds[i] = edges[i];
    neg[i] = ng[i];
  }
  for (int i = 0; i + 1 < nb; ++i) {
    counts[i] = ng[i + 1] - ng[i];
    if (m0) m0[i] = fb_m0_rule(counts[i]);
  }
  if (n_inertia) *n_inertia = ir.evals;
  return 0;
}
