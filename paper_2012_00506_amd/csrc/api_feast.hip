// C ABI: feast_band_slice -- FEAST on band slices (Algorithm alg:FEAST of
// Section 2.2 with the slice count check of Section 3.2).
#include <math.h>

#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <numeric>
#include <vector>

#include "chol64.h"
#include "rr.h"
#include "solve_job.h"
#include "prof.h"

namespace fb {

// ---------------------------------------------------------------- quadrature
// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton's method
// on the Legendre polynomial P_k (three-term recurrence), weights
// 2 / ((1 - x^2) P_k'(x)^2).
void gauss_legendre(int k, std::vector<double>& x, std::vector<double>& w) {
  x.assign(k, 0.0);
  w.assign(k, 0.0);
  for (int i = 0; i < (k + 1) / 2; ++i) {
    double r = cos(M_PI * (i + 0.75) / (k + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int j = 2; j <= k; ++j) {
        double p2 = ((2.0 * j - 1.0) * r * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (k == 1) {
        p1 = r;
        p0 = 1.0;
      }
      dp = k * (r * p1 - p0) / (r * r - 1.0);
      double dr = p1 / dp;
      r -= dr;
      if (fabs(dr) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = r;
      for (int j = 2; j <= k; ++j) {
        double p2 = ((2.0 * j - 1.0) * r * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (k == 1) p0 = 1.0;
      dp = k * (r * p1 - p0) / (r * r - 1.0);
    }
    double wt = 2.0 / ((1.0 - r * r) * dp * dp);
    x[k - 1 - i] = r;
    w[k - 1 - i] = wt;
    x[i] = -r;
    w[i] = wt;
  }
}

// Descending Landen (arithmetic-geometric mean) chain of modulus k with
// complementary modulus kc = sqrt(1 - k^2), given separately because 1 - k^2
// cancels for k near 1: a_0 = 1, b_0 = kc, c_0 = k; a_{i+1} = (a_i + b_i)/2,
// b_{i+1} = sqrt(a_i b_i), c_{i+1} = (a_i - b_i)/2.  K(k) = pi / (2 a_N).
struct LandenChain {
  double a[48], c[48];
  int n = 0;
};

static LandenChain landen(double k, double kc) {
  LandenChain g;
  g.a[0] = 1.0;
  g.c[0] = k;
  double b = kc;
  while (g.n < 47 && fabs(g.c[g.n]) > 4e-16 * g.a[g.n]) {
    const double an = g.a[g.n];
    g.a[g.n + 1] = 0.5 * (an + b);
    g.c[g.n + 1] = 0.5 * (an - b);
    b = sqrt(an * b);
    ++g.n;
  }
  return g;
}

// Jacobi sn, cn, dn of argument u on the chain: phi_N = 2^N a_N u,
// phi_{i-1} = (phi_i + asin(c_i sin(phi_i) / a_i)) / 2, sn = sin phi_0,
// cn = cos phi_0, dn = cn / cos(phi_1 - phi_0)
static void jacobi_sncndn(double u, const LandenChain& g, double* sn, double* cn, double* dn) {
  double phi = ldexp(g.a[g.n] * u, g.n), phi1 = phi;
  for (int i = g.n; i >= 1; --i) {
    phi1 = phi;
    phi = 0.5 * (phi + asin(g.c[i] * sin(phi) / g.a[i]));
  }
  *sn = sin(phi);
  *cn = cos(phi);
  *dn = g.n > 0 ? *cn / cos(phi1 - phi) : 1.0;
}

// Zolotarev filter on the scaled slice t in (-1, 1) with inner fraction b:
// Z(x) = M x prod_{j<m}(x^2 + c_{2j}) / prod_{j<=m}(x^2 + c_{2j-1}), the best
// type (2m-1, 2m) approximation of sign(x) on [-1, -l] U [l, 1] with
// c_j = l^2 sn^2 / cn^2 (j K'/(2m); k'), k' = sqrt(1 - l^2),
// l = ((1 - b)/(1 + b))^2; M centres the error, whose extrema on [l, 1] are at
// x = l / dn(j K'/(2m); k').  With x = s (1 + t)/(1 - t), s = sqrt(l), the
// filter (1 + Z(x(t)))/2 has its poles t_q = (i a - s)/(i a + s),
// a = sqrt(c_{2q-1}), on the unit circle; its pole part gives
// w_q = -rho_q s ((s^2 - a^2) - 2 i a s) / (a^2 + s^2)^2 with rho_q the residue
// of Z at x = i a.  The constant (1 + Z(-s))/2, below half the error, is left
// out so that the filter keeps the form sum_q 2 Re[w_q / (t_q - t)].
static void zolotarev_nodes(int m, double b, std::vector<c128>& t, std::vector<c128>& w) {
  const double l = ((1.0 - b) / (1.0 + b)) * ((1.0 - b) / (1.0 + b));
  const double s = sqrt(l);
  const LandenChain g = landen(sqrt((1.0 - l) * (1.0 + l)), l);
  const double Kp = M_PI / (2.0 * g.a[g.n]);
  std::vector<double> c(2 * m, 0.0);  // c[1..2m-1]
  double sn, cn, dn;
  for (int j = 1; j < 2 * m; ++j) {
    jacobi_sncndn(j * Kp / (2.0 * m), g, &sn, &cn, &dn);
    c[j] = l * l * (sn * sn) / (cn * cn);
  }
  auto zt = [&](double x) {
    double num = x, den = 1.0;
    for (int j = 1; j < m; ++j) num *= x * x + c[2 * j];
    for (int j = 1; j <= m; ++j) den *= x * x + c[2 * j - 1];
    return num / den;
  };
  jacobi_sncndn(Kp / (2.0 * m), g, &sn, &cn, &dn);
  const double M = 2.0 / (zt(l) + zt(l / dn));
  t.resize(m);
  w.resize(m);
  for (int q = 1; q <= m; ++q) {
    const double a2 = c[2 * q - 1], a = sqrt(a2);
    double num = M, den = 2.0;
    for (int j = 1; j < m; ++j) num *= c[2 * j] - a2;
    for (int j = 1; j <= m; ++j)
      if (j != q) den *= c[2 * j - 1] - a2;
    const double rho = num / den, d = a2 + l;
    t[q - 1] = mk((a2 - l) / d, 2.0 * a * s / d);
    w[q - 1] = mk(-rho * s * (l - a2) / (d * d), 2.0 * rho * l * a / (d * d));
  }
}

// Nodes and weights on the upper half of the contour through the slice ends,
// z(t) = c + r (cos t + i rho sin t) (rho = 1: the circle), for
// P = (1/(2 pi i)) \oint (zI - B)^{-1} dz with the lower half by conjugation:
// w_j = (dt_j / (2 pi)) z'(t_j) / i = (dt_j / (2 pi)) r (rho cos t_j + i sin t_j).
// rule 0: Gauss-Legendre in t on [0, pi], t_j = (pi/2)(1 - x_j),
// dt_j = (pi/2) omega_j, so w_j = (omega_j / 4) r (rho cos t_j + i sin t_j);
// rule 1: midpoint angles t_j = pi (j + 1/2) / k, dt_j = pi / k;
// rule 2: the Zolotarev filter with inner fraction ratio, mapped to the slice.
void contour(double lo, double hi, int k, int rule, double ratio, std::vector<c128>& z,
             std::vector<c128>& w) {
  double c = 0.5 * (lo + hi), r = 0.5 * (hi - lo);
  if (rule == 2) {
    zolotarev_nodes(k, ratio, z, w);
    for (int j = 0; j < k; ++j) {
      z[j] = mk(c + r * z[j].x, r * z[j].y);
      w[j] = mk(r * w[j].x, r * w[j].y);
    }
    return;
  }
  const double rho = ratio > 0.0 ? ratio : 1.0;
  std::vector<double> x, om;
  if (rule == 0) gauss_legendre(k, x, om);
  z.resize(k);
  w.resize(k);
  for (int j = 0; j < k; ++j) {
    const double th = rule == 0 ? 0.5 * M_PI * (1.0 - x[j]) : M_PI * (j + 0.5) / k;
    const double f = rule == 0 ? 0.25 * om[j] : 0.5 / k;  // dt_j / (2 pi)
    const double ct = cos(th), st = sin(th);
    z[j] = mk(c + r * ct, r * rho * st);
    w[j] = mk(f * r * rho * ct, f * r * st);
  }
}

// rule and ratio as fb_feast_opts takes them
static bool contour_ok(int rule, double ratio) {
  if (rule == 0 || rule == 1) return ratio >= 0.0 && isfinite(ratio);
  if (rule == 2) return ratio > 0.0 && ratio < 1.0;
  return false;
}

// Captured filter sweeps, keyed by every argument that shapes their launches
// (pointers, sizes, options; node values and job tables are uploaded before
// each replay).  Process-wide, guarded by a mutex, at most kMaxGraphs of them:
// the oldest is destroyed first (a replay still in flight completes; HIP frees
// an executable graph once its launches end).
constexpr size_t kMaxGraphs = 64;
static std::mutex g_graph_mu;
struct GraphCache {
  std::map<std::string, hipGraphExec_t> by_key;
  std::vector<std::string> order;
};
static GraphCache& graph_cache() {
  static GraphCache c;
  return c;
}
// Launches the sweep cached under k; false when there is none.
static bool graph_launch(const std::string& k, hipStream_t st, hipError_t* err) {
  std::lock_guard<std::mutex> g(g_graph_mu);
  auto it = graph_cache().by_key.find(k);
  if (it == graph_cache().by_key.end()) return false;
  *err = hipGraphLaunch(it->second, st);
  return true;
}
// Caches a newly instantiated sweep under k and launches it.
static hipError_t graph_store_launch(const std::string& k, hipGraphExec_t e, hipStream_t st) {
  std::lock_guard<std::mutex> g(g_graph_mu);
  GraphCache& c = graph_cache();
  auto it = c.by_key.find(k);
  if (it != c.by_key.end()) {  // another thread captured the same sweep meanwhile
    (void)hipGraphExecDestroy(e);
    return hipGraphLaunch(it->second, st);
  }
  while (c.order.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(c.by_key[c.order.front()]);
    c.by_key.erase(c.order.front());
    c.order.erase(c.order.begin());
  }
  c.by_key[k] = e;
  c.order.push_back(k);
  return hipGraphLaunch(e, st);
}

// Loads a tuning file named in the options once per process (false when it
// cannot be read).
static bool tune_cache_ok(const char* path) {
  if (!path) return true;
  static std::mutex mu;
  static std::set<std::string> loaded;
  std::lock_guard<std::mutex> g(mu);
  if (loaded.count(path)) return true;
  if (fb_tune_load(path) < 0) return false;
  loaded.insert(path);
  return true;
}

struct SliceBufs {
  c128 *Y, *Q, *X;      // n x m0 each (start block, filter sum, scratch)
  c128 *G, *V, *W;      // m0 x m0
  c128 *Dinv, *Pb;      // Cholesky: diagonal-block inverses, panel scratch (m0 x 64 each)
  c128* gpart;          // split partial sums of the long products
  double *s, *lam, *res, *scale, *part, *cscale;
  int32_t *order, *idx, *kept, *sweeps, *cinfo;
};

// Pivots r_jj^2 of the equilibrated Gram matrices at or below this end the
// Cholesky QR of a slice (the eigen-decomposition passes take over).
constexpr double kCholPivMin = 1e-12;
// Most split ranges of a long A^H B product (partial sums kept per slice).
constexpr int kMaxSplit = 8;

// C = op(A) B descriptors of the orthonormalisation and Rayleigh-Ritz
// products (all complex128, column-major).
static GemmProb gp_tn(const c128* A, int64_t lda, const c128* B, int64_t ldb, c128* C,
                      int64_t ldc, int M, int N, int K, int herm) {
  GemmProb p{};
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;
  p.M = M;
  p.N = N;
  p.K = K;
  p.transa = 1;
  p.herm = herm;
  p.alpha = mk(1.0, 0.0);
  p.ksplit = 1;
  return p;
}
static GemmProb gp_nn(const c128* A, int64_t lda, const c128* B, int64_t ldb, c128* C,
                      int64_t ldc, int M, int N, int K, int b_upper) {
  GemmProb p = gp_tn(A, lda, B, ldb, C, ldc, M, N, K, 0);
  p.transa = 0;
  p.b_upper = b_upper;
  return p;
}

static GemmProb with_part(GemmProb p, c128* part) {
  p.part = part;
  return p;
}

static JacobiJob jacobi_job(const SliceBufs& b, int m, double* w) {
  JacobiJob J{};
  J.m = m;
  J.A = b.G;
  J.lda = m;
  J.V = b.V;
  J.ldv = m;
  J.W = b.W;
  J.ldw = m;
  J.w = w;
  J.order = b.order;
  J.sweeps = b.sweeps;
  return J;
}

// k_colscale: s_j = 1 / sqrt(Re G_jj); k_equil: G_ij *= s_i s_j (upper
// triangle).  A zero or non-finite column makes the scaled matrix non-finite,
// which the Cholesky pivot test then rejects.
__global__ void k_colscale(const CholProb* __restrict__ probs) {
  const CholProb P = probs[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.m) return;
  const double d = gld(P.G + (int64_t)j * P.ld + j).x;
  gst(const_cast<double*>(P.rowscale) + j, 1.0 / sqrt(d));
}
__global__ void __launch_bounds__(256) k_equil(const CholProb* __restrict__ probs) {
  const CholProb P = probs[blockIdx.y];
  const int m = P.m;
  const int64_t tot = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    if (i > j) continue;
    c128* g = P.G + (int64_t)j * P.ld + i;
    gst(g, (gld(P.rowscale + i) * gld(P.rowscale + j)) * gld(g));
  }
}

// Q_i = sum_j w_ij (z_ij - B)^{-1} Y_i (+ conj(w_ij) (z_ij - B)^{-H} Y_i) for
// the slices in act.  The (node, direction) pairs are taken in order, P of
// them per batched launch over all slices (batched) or one pair of one slice
// per launch (plain); each pair's solutions go to their own buffer
// Xp[i * P + p] and are then added into Q_i in pair order, so the sum does
// not depend on how the pairs were grouped.
// Solve jobs and accumulation jobs of the pairs p0 .. p0+np-1 for the active
// slices (all of them, or only act[only] when only >= 0).
template <typename R>
void build_pair_jobs(int64_t n, int tile, int ne, const std::vector<int>& act, const int32_t* m,
                     c128* const* Yc, const int64_t* ldyc, c128* const* Qc, const int64_t* ldqc,
                     c128* const* Xp, int P, const std::vector<std::pair<int, int>>& pairs, int p0,
                     int np, int only, const std::vector<c128>& wsys, bool cplx,
                     std::vector<SolveJob>& jobs, std::vector<AccJob>& aj, int& maxm) {
  jobs.clear();
  aj.clear();
  maxm = 0;
  for (int p = 0; p < np; ++p) {
    const int j = pairs[p0 + p].first, dir = pairs[p0 + p].second;
    for (size_t a = 0; a < act.size(); ++a) {
      if (only >= 0 && (int)a != only) continue;
      const int i = act[a];
      for (int c0 = 0; c0 < m[i]; c0 += tile) {
        SolveJob jb{};
        jb.sys = i * ne + j;
        jb.dir = dir;
        jb.col0 = c0;
        jb.ncol = std::min(tile, m[i] - c0);
        jb.in = Yc[i];
        jb.ldin = ldyc[i];
        jb.mid = Xp[(size_t)i * P + p];
        jb.out = Xp[(size_t)i * P + p];
        jb.ldout = n;
        jb.ldmid = n * (int64_t)(sizeof(c128) / sizeof(cx<R>));
        jobs.push_back(jb);
      }
    }
  }
  for (size_t a = 0; a < act.size(); ++a) {
    if (only >= 0 && (int)a != only) continue;
    const int i = act[a];
    AccJob J{};
    J.Q = Qc[i];
    J.ldq = ldqc[i];
    J.ldx = n;
    J.np = np;
    J.m = m[i];
    J.acc_real = cplx ? 0 : 1;
    J.init = p0 == 0;  // the first pairs of the sum write Q
    for (int p = 0; p < np; ++p) {
      const int j = pairs[p0 + p].first, dir = pairs[p0 + p].second;
      J.X[p] = Xp[(size_t)i * P + p];
      const c128 w = wsys[i * ne + j];
      J.w[p] = dir == 0 ? w : cconj(w);
    }
    maxm = std::max(maxm, m[i]);
    aj.push_back(J);
  }
}

static std::vector<std::pair<int, int>> node_pairs(int ne, bool cplx) {
  std::vector<std::pair<int, int>> pairs;
  for (int j = 0; j < ne; ++j)
    for (int dir = 0; dir < (cplx ? 2 : 1); ++dir) pairs.push_back({j, dir});
  return pairs;
}

template <typename R>
int filter_apply(const Band& bd, const FactorBufs<R>& f, int ne, const std::vector<int>& act,
                 const int32_t* m, c128* const* Yc, const int64_t* ldyc, c128* const* Qc,
                 const int64_t* ldqc, c128* const* Xp, int P, AccJob* acc_dev,
                 const std::vector<c128>& zsys, const std::vector<c128>& wsys, bool cplx,
                 bool batched, bool ir, double ir_tol, int ir_max, bool need_res, RefineBufs& rb,
                 std::vector<double>& sys_res, std::vector<int32_t>& sys_pass, int* unconverged,
                 hipStream_t st, const C128Fallback* fb) {
  const int64_t n = bd.n;
  const std::vector<std::pair<int, int>> pairs = node_pairs(ne, cplx);
  const int npair = (int)pairs.size();
  const int chunk = batched ? std::max(1, std::min(P, npair)) : 1;
  if (chunk > kMaxPairs) return FB_ERR_INTERNAL;
  const size_t groups = batched ? 1 : act.size();
  std::vector<SolveJob> jobs;
  std::vector<AccJob> aj;
  for (size_t g = 0; g < groups; ++g)
    for (int p0 = 0; p0 < npair; p0 += chunk) {
      const int np = std::min(chunk, npair - p0);
      int maxm = 0;
      build_pair_jobs<R>(n, rb.tile, ne, act, m, Yc, ldyc, Qc, ldqc, Xp, P, pairs, p0, np,
                         batched ? -1 : (int)g, wsys, cplx, jobs, aj, maxm);
      FB_TRY(solve_refine<R>(bd, f.mats, f.matsT, f.perm, jobs, zsys, ir, ir_tol, ir_max, need_res, rb,
                             sys_res, sys_pass, unconverged, st, fb));
      FB_HIP(hipMemcpyAsync(acc_dev, aj.data(), sizeof(AccJob) * aj.size(), hipMemcpyHostToDevice, st));
      FB_TRY(accumulate_pairs(acc_dev, (int)aj.size(), n, maxm, st));
    }
  return 0;
}

// Pairs per batched launch: as many (node, direction) pairs as the budget
// leaves room for, each needing one n x m complex128 buffer per slice.
static int pairs_per_launch(double budget, int fixed, bool batched, int npair, size_t base,
                            size_t per_pair) {
  if (!batched || npair <= 1) return 1;
  if (fixed > 0) return std::min(fixed, std::min(npair, kMaxPairs));
  if (!(budget > 0)) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
    budget = 0.5 * (double)tot;
  }
  const double room = budget - (double)base;
  int p = per_pair ? (int)std::min<double>(npair, floor(room / (double)per_pair)) : npair;
  return std::max(1, std::min(p, std::min(npair, kMaxPairs)));
}

// Workspace of one wave of slices: W slots of m0 <= maxm each.
template <typename R>
struct FeastBufs {
  FactorBufs<R> f;
  double* shifts = nullptr;
  int32_t* cnt = nullptr;
  void* iscratch = nullptr;
  std::vector<SliceBufs> sb;
  JacobiJob* jj_dev = nullptr;
  EigWork ew;
  int32_t* perm_dev = nullptr;
  AccJob* acc_dev = nullptr;
  int tile = 16, P = 1;
  std::vector<c128*> Xp;  // slot * P + pair
  RefineBufs rb;
  FactorBufs<double> f64fb;       // complex128 fallback factors (precision 1)
  C128Fallback fb;
  CholProb* chol_dev = nullptr;  // W descriptors
  GemmProb* gdev = nullptr;      // gcap descriptors
  size_t gcap = 0;
  int kmax = 1;                  // split ranges the partial buffers hold
};

static int gram_tiles(int m) {
  const int t = (m + kGemmTile - 1) / kGemmTile;
  return t * (t + 1) / 2;
}

// The long products (contraction over the n rows of the basis) of one
// batch, split so that the batch has about 1024 workgroups.
template <typename R>
int run_gram(std::vector<GemmProb>& g, const FeastBufs<R>& fb, hipStream_t st) {
  if (g.empty()) return 0;
  long tiles = 0;
  for (const GemmProb& p : g) tiles += gram_tiles(p.M);
  const int k = (int)std::max<long>(1, std::min<long>(fb.kmax, (1024 + tiles - 1) / tiles));
  for (GemmProb& p : g) p.ksplit = p.part ? k : 1;
  return gemm_batched(g, fb.gdev, st);
}

static CholProb chol_prob(const SliceBufs& b, int m, c128* T, bool scale) {
  CholProb c{};
  c.G = b.G;
  c.ld = m;
  c.T = T;
  c.ldt = m;
  c.Dinv = b.Dinv;
  c.P = b.Pb;
  c.rowscale = scale ? b.cscale : nullptr;
  c.info = b.cinfo;
  c.m = m;
  return c;
}

template <typename R>
int equilibrate(const std::vector<CholProb>& cp, const FeastBufs<R>& fb, hipStream_t st) {
  if (cp.empty()) return 0;
  int mmax = 1;
  for (const CholProb& c : cp) mmax = std::max(mmax, c.m);
  FB_HIP(hipMemcpyAsync(fb.chol_dev, cp.data(), sizeof(CholProb) * cp.size(),
                        hipMemcpyHostToDevice, st));
  k_colscale<<<dim3((mmax + 255) / 256, (unsigned)cp.size()), 256, 0, st>>>(fb.chol_dev);
  FB_HIP(hipGetLastError());
  const int grid = (int)std::min<int64_t>(((int64_t)mmax * mmax + 255) / 256, 4096);
  k_equil<<<dim3(grid, (unsigned)cp.size()), 256, 0, st>>>(fb.chol_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

template <typename R>
void carve_feast(Arena& ar, const Band& bd, int W, int maxm, int ne, bool ir, int P,
                 FeastBufs<R>& fb) {
  const int64_t n = bd.n;
  carve_factors<R>(ar, bd, W * ne, fb.f);
  if (ir && ne > 0) {
    fb.fb.cap = feast_fallback_cap(W * ne);
    carve_factors<double>(ar, bd, fb.fb.cap, fb.f64fb);
    fb.fb.f = &fb.f64fb;
  }
  fb.shifts = ar.take<double>(2 * W);
  fb.cnt = ar.take<int32_t>(6 * W);
  size_t iscr = inertia_scratch_bytes(bd, 2 * W);
  fb.iscratch = iscr ? (void*)ar.take<char>(iscr) : nullptr;
  fb.sb.assign(W, SliceBufs{});
  const int m = maxm;
  for (int a = 0; a < W; ++a) {
    SliceBufs& b = fb.sb[a];
    b.Y = ar.take<c128>((size_t)n * m);
    b.Q = ar.take<c128>((size_t)n * m);
    b.X = ar.take<c128>((size_t)n * m);
    b.G = ar.take<c128>((size_t)m * m);
    b.V = ar.take<c128>((size_t)m * m);
    b.W = ar.take<c128>((size_t)m * m);
    b.s = ar.take<double>(m);
    b.lam = ar.take<double>(m);
    b.res = ar.take<double>(m);
    b.scale = ar.take<double>(m);
    b.part = ar.take<double>(eig_resid_part_doubles(n, m));
    b.order = ar.take<int32_t>(m);
    b.idx = ar.take<int32_t>(m);
    b.kept = ar.take<int32_t>(1);
    b.sweeps = ar.take<int32_t>(1);
    const size_t nblk = (size_t)(m + kGemmTile - 1) / kGemmTile;
    b.Dinv = ar.take<c128>(nblk * kGemmTile * kGemmTile);
    b.Pb = ar.take<c128>((size_t)m * kGemmTile);
    b.cscale = ar.take<double>(m);
    b.cinfo = ar.take<int32_t>(1);
  }
  fb.kmax = std::max(1, std::min(kMaxSplit, (1024 + gram_tiles(m) - 1) / gram_tiles(m)));
  for (int a = 0; a < W; ++a)
    fb.sb[a].gpart = fb.kmax > 1 ? ar.take<c128>((size_t)fb.kmax * m * m) : nullptr;
  fb.chol_dev = ar.take<CholProb>(W);
  fb.gcap = std::max(chol_gemm_descs(W, m), (size_t)kGemmMaxProbs);
  fb.gdev = ar.take<GemmProb>(fb.gcap);
  fb.jj_dev = ar.take<JacobiJob>(W);
  carve_eig_work(ar, std::vector<int>(W, maxm), fb.ew);
  fb.perm_dev = ar.take<int32_t>(maxm);
  fb.acc_dev = ar.take<AccJob>(W);
  fb.tile = solve_tile<R>(bd.b);
  const int max_jobs = W * ((maxm + fb.tile - 1) / fb.tile);
  fb.P = P;
  fb.Xp.assign((size_t)W * P, nullptr);
  for (int a = 0; a < W; ++a) {
    fb.Xp[(size_t)a * P] = fb.sb[a].X;
    for (int p = 1; p < P; ++p) fb.Xp[(size_t)a * P + p] = ar.take<c128>((size_t)n * m);
  }
  carve_refine(ar, bd, fb.tile, max_jobs * P, ir, ir, fb.rb);
}

// Orthonormalisation and Rayleigh-Ritz of the filtered blocks of the slots
// in act (Algorithm alg:FEAST): on entry sb[i].Q holds the n x m0[i] block;
// on exit sb[i].Q holds the orthonormal basis (kept[i] columns), sb[i].X the
// Ritz vectors, sb[i].lam the Ritz values (ascending) and sb[i].res their
// residuals ||B x - lambda x||_2 / ||B||_1; sb[i].Y is scratch (its columns
// from kept[i] on are left as they were).  path[i]: 0 Cholesky QR twice,
// 1 the eigen-decomposition passes.
template <typename R>
int ortho_rr(const Band& bd, int nslice, const std::vector<int>& act, const int32_t* m0,
             std::vector<int>& kept, std::vector<int>& path, FeastBufs<R>& fbuf, hipStream_t st) {
  const int64_t n = bd.n;
  std::vector<SliceBufs>& sb = fbuf.sb;
  JacobiJob* jj_dev = fbuf.jj_dev;
  const EigWork& ew = fbuf.ew;
  // ---- orthonormalise: Cholesky QR twice on the column-equilibrated block
  // (D scales every column of Q to unit norm): G = D Q^H Q D = R1^H R1,
  // Q1 = Q D R1^{-1}; Q1^H Q1 = R2^H R2, Q2 = Q1 R2^{-1}.  It applies when
  // every pivot r_jj^2 of both factorisations is above kCholPivMin (the
  // equilibrated Gram matrix has unit diagonal, and r_jj is the sine of the
  // angle between column j and the columns before it); slices where it
  // does not fall back to the two eigen-decomposition passes below.
  std::vector<int> chol_ok(nslice, 0), eig_path;
  {
    std::vector<GemmProb> g;
    for (int i : act)
      g.push_back(with_part(gp_tn(sb[i].Q, n, sb[i].Q, n, sb[i].G, m0[i], m0[i], m0[i], (int)n, 1),
                            sb[i].gpart));
    FB_TRY(run_gram(g, fbuf, st));
    std::vector<CholProb> cp;
    for (int i : act) cp.push_back(chol_prob(sb[i], m0[i], sb[i].V, true));
    FB_TRY(equilibrate(cp, fbuf, st));
    FB_TRY(chol_inverse(cp, fbuf.chol_dev, fbuf.gdev, fbuf.gcap, kCholPivMin, st));
    g.clear();  // Q1 = Q (D R1^{-1}) into X
    for (int i : act) g.push_back(gp_nn(sb[i].Q, n, sb[i].V, m0[i], sb[i].X, n, (int)n, m0[i],
                                        m0[i], 1));
    FB_TRY(gemm_batched(g, fbuf.gdev, st));
    std::vector<int32_t> inf1(nslice, 0);
    for (int i : act) FB_HIP(hipMemcpyAsync(&inf1[i], sb[i].cinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    std::vector<int> pass2;
    for (int i : act) (inf1[i] == 0 ? pass2 : eig_path).push_back(i);
    g.clear();
    for (int i : pass2)
      g.push_back(with_part(gp_tn(sb[i].X, n, sb[i].X, n, sb[i].G, m0[i], m0[i], m0[i], (int)n, 1),
                            sb[i].gpart));
    FB_TRY(run_gram(g, fbuf, st));
    cp.clear();
    for (int i : pass2) cp.push_back(chol_prob(sb[i], m0[i], sb[i].V, false));
    FB_TRY(chol_inverse(cp, fbuf.chol_dev, fbuf.gdev, fbuf.gcap, kCholPivMin, st));
    std::vector<int32_t> inf2(nslice, 0);
    for (int i : pass2) FB_HIP(hipMemcpyAsync(&inf2[i], sb[i].cinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    g.clear();  // Q2 = Q1 R2^{-1} into Q (the filter sum is spent)
    for (int i : pass2) {
      if (inf2[i] != 0) {
        eig_path.push_back(i);
        continue;
      }
      chol_ok[i] = 1;
      kept[i] = m0[i];
      g.push_back(gp_nn(sb[i].X, n, sb[i].V, m0[i], sb[i].Q, n, (int)n, m0[i], m0[i], 1));
    }
    FB_TRY(gemm_batched(g, fbuf.gdev, st));
  }
  // ---- fallback, pass 1: Q^H Q = V s V^H; Q V over every eigenvector,
  // each column's norm measured on the product, the columns above 1e-12 of
  // the largest kept and scaled to unit norm.  The Gram matrix of a filtered
  // block spans more orders of magnitude than FP64 resolves: its smallest s
  // are rounding noise (often negative) while the directions Q v formed from
  // Q are still accurate, and they carry the last digits of the wanted
  // eigenvectors (dropping those whose computed s is at or below eps max s
  // stalls the residuals near 1e-10 under a 16-node filter).  The rank
  // decision, s > 1e-14 max s, is taken in pass 2 on the well-scaled block.
  std::sort(eig_path.begin(), eig_path.end());
  if (!eig_path.empty()) {
    std::vector<JacobiJob> jj;
    std::vector<GemmProb> g;
    for (int i : eig_path) {
      int m = m0[i];
      g.push_back(with_part(gp_tn(sb[i].Q, n, sb[i].Q, n, sb[i].G, m, m, m, (int)n, 2), sb[i].gpart));
      jj.push_back(jacobi_job(sb[i], m, sb[i].s));
    }
    FB_TRY(run_gram(g, fbuf, st));
    FB_TRY(reduced_eig(jj, jj_dev, ew, 60, 1e-14, st));
    g.clear();
    for (int i : eig_path)  // Q V into X
      g.push_back(gp_nn(sb[i].Q, n, sb[i].W, m0[i], sb[i].X, n, (int)n, m0[i], m0[i], 0));
    FB_TRY(gemm_batched(g, fbuf.gdev, st));
    for (int i : eig_path)  // column norms into s
      FB_TRY(col_norm_keep(sb[i].X, n, n, m0[i], 1e-12, sb[i].s, sb[i].idx, sb[i].scale,
                           sb[i].kept, st));
    for (int i : eig_path)
      FB_HIP(hipMemcpyAsync(&kept[i], sb[i].kept, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    std::vector<int> prev_kept(kept);
    jj.clear();
    g.clear();
    for (int i : eig_path) {
      int k = kept[i];
      if (k <= 0) continue;
      // Q' = kept columns of Q V at unit norm, into Q (the filter sum is spent)
      FB_TRY(gather_cols(sb[i].X, n, false, sb[i].Q, n, n, k, sb[i].idx, sb[i].scale, st));
      // pass 2: Q'^H Q' = I + E with E growing with the spread of s;
      // orthonormalising Q' once more makes the basis orthonormal to
      // rounding, which the eigen-residual floor needs
      g.push_back(with_part(gp_tn(sb[i].Q, n, sb[i].Q, n, sb[i].G, k, k, k, (int)n, 2), sb[i].gpart));
      jj.push_back(jacobi_job(sb[i], k, sb[i].s));
    }
    FB_TRY(run_gram(g, fbuf, st));
    if (!jj.empty()) FB_TRY(reduced_eig(jj, jj_dev, ew, 60, 1e-14, st));
    for (int i : eig_path)
      if (kept[i] > 0)
        FB_TRY(gram_keep(sb[i].s, kept[i], 1e-14, sb[i].idx, sb[i].scale, sb[i].kept, st));
    for (int i : eig_path)
      if (kept[i] > 0)
        FB_HIP(hipMemcpyAsync(&kept[i], sb[i].kept, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    g.clear();
    for (int i : eig_path) {
      int k = kept[i];
      if (k <= 0) continue;
      // Q'' = Q' W2[:, idx] diag(scale) into X, which then trades places with Q
      const int k1 = (int)prev_kept[i];
      FB_TRY(gather_cols(sb[i].W, k1, false, sb[i].V, k1, k1, k, sb[i].idx, sb[i].scale, st));
      g.push_back(gp_nn(sb[i].Q, n, sb[i].V, k1, sb[i].X, n, (int)n, k, k1, 0));
    }
    FB_TRY(gemm_batched(g, fbuf.gdev, st));
    for (int i : eig_path)
      if (kept[i] > 0) std::swap(sb[i].Q, sb[i].X);
  }
  // ---- Rayleigh-Ritz: A_q = Q^H B Q, A_q W = W Lambda, X = Q W
  {
    std::vector<JacobiJob> jj;
    std::vector<GemmProb> g;
    for (int i : act) {
      int k = kept[i];
      if (k <= 0) continue;
      // B Q into Y (its trailing columns keep the start vectors)
      FB_TRY(band_matmul(bd, sb[i].Q, n, sb[i].Y, n, k, st));
      g.push_back(with_part(gp_tn(sb[i].Q, n, sb[i].Y, n, sb[i].G, k, k, k, (int)n, 2), sb[i].gpart));
      jj.push_back(jacobi_job(sb[i], k, sb[i].lam));
    }
    FB_TRY(run_gram(g, fbuf, st));
    if (!jj.empty()) FB_TRY(reduced_eig(jj, jj_dev, ew, 60, 1e-14, st));
    g.clear();
    for (int i : act) {  // Ritz vectors X = Q W into X
      int k = kept[i];
      if (k > 0) g.push_back(gp_nn(sb[i].Q, n, sb[i].W, k, sb[i].X, n, (int)n, k, k, 0));
    }
    FB_TRY(gemm_batched(g, fbuf.gdev, st));
  }
  for (int i : act) {
    path[i] = chol_ok[i] ? 0 : 1;
    if (kept[i] > 0)
      FB_TRY(eig_residuals(bd, sb[i].X, n, sb[i].lam, kept[i], sb[i].part, sb[i].res, st));
  }
  return 0;
}

// FEAST on nslice slices that share one wave's workspace.
template <typename R>
int feast_wave(const Band& bd, int nslice, const double* lo, const double* hi, const int32_t* m0,
               const int32_t* m_expected, void* const* Y, const int64_t* ldy,
               double* const* evals, double* const* resid, int32_t* m_found, int32_t* iters,
               int32_t* info, const fb_feast_opts* o, FeastBufs<R>& fbuf, hipStream_t st) {
  const bool ir = o->precision == 1;
  const int ne = o->n_nodes;
  const int64_t n = bd.n;
  const bool cplx = bd.cplx;
  const int nsys = nslice * ne;
  FactorBufs<R>& f = fbuf.f;
  double* shifts = fbuf.shifts;
  int32_t* cnt = fbuf.cnt;
  void* iscratch = fbuf.iscratch;
  std::vector<SliceBufs>& sb = fbuf.sb;
  JacobiJob* jj_dev = fbuf.jj_dev;
  const EigWork& ew = fbuf.ew;
  int32_t* perm_dev = fbuf.perm_dev;
  AccJob* acc_dev = fbuf.acc_dev;
  const int P = fbuf.P;
  std::vector<c128*>& Xp = fbuf.Xp;
  RefineBufs& rb = fbuf.rb;

  // ---- exact counts (Sylvester inertia at the slice ends)
  double stats[3];
  FB_TRY(band_stats_host(bd, stats, st));
  std::vector<int> mexp(nslice);
  if (m_expected) {
    for (int i = 0; i < nslice; ++i) mexp[i] = m_expected[i];
  } else {
    std::vector<double> sh(2 * nslice);
    for (int i = 0; i < nslice; ++i) {
      sh[2 * i] = lo[i];
      sh[2 * i + 1] = hi[i];
    }
    FB_HIP(hipMemcpyAsync(shifts, sh.data(), sizeof(double) * 2 * nslice, hipMemcpyHostToDevice, st));
    FB_TRY(launch_inertia(bd, 2 * nslice, shifts, cnt, iscratch, st));
    std::vector<int32_t> h(6 * nslice);
    FB_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * 6 * nslice, hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < nslice; ++i) mexp[i] = h[6 * i + 3] - h[6 * i];
  }

  // ---- nodes, weights and the factorisations of every (slice, node)
  std::vector<c128> zsys(nsys), wsys(nsys);
  std::vector<double> zh(2 * nsys);
  for (int i = 0; i < nslice; ++i) {
    std::vector<c128> z, w;
    contour(lo[i], hi[i], ne, o->rule, o->ratio, z, w);
    for (int j = 0; j < ne; ++j) {
      zsys[i * ne + j] = z[j];
      wsys[i * ne + j] = w[j];
      zh[2 * (i * ne + j)] = z[j].x;
      zh[2 * (i * ne + j) + 1] = z[j].y;
    }
  }
  FB_TRY(factor_systems<R>(bd, nsys, zh.data(), f, st));
  fbuf.fb.reset();  // new shifts: no complex128 factors carry over

  // ---- start blocks
  std::vector<int> done(nslice, 0), kept(nslice, 0), good(nslice, 0), inside(nslice, 0);
  std::vector<int> fellback(nslice, 0);  // a system of the slice fell back to complex128
  std::vector<std::vector<double>> hl(nslice), hr(nslice);
  for (int i = 0; i < nslice; ++i) {
    iters[i] = 0;
    m_found[i] = 0;
    info[i] = 0;
    if (m0[i] < mexp[i]) {
      info[i] = 5;
      done[i] = 1;
      continue;
    }
    FB_TRY(gather_cols(Y[i], ldy[i], !cplx, sb[i].Y, n, n, m0[i], nullptr, nullptr, st));
  }

  std::vector<double> sys_res(nsys, 0.0);
  std::vector<int32_t> sys_pass(nsys, 0);
  std::vector<SolveJob> jobs;
  // complex64 solves without refinement while a slice is far from converged
  // (its eigen-residuals, computed in FP64, decide; at most kCoarseIters
  // iterations): they move the subspace as far as refined ones there
  constexpr int kCoarseIters = 3;
  std::vector<int> coarse(nslice, ir && o->ir_from > 0 ? 1 : 0), ncoarse(nslice, 0);
  for (int it = 1; it <= o->max_iter; ++it) {
    std::vector<int> act;
    for (int i = 0; i < nslice; ++i)
      if (!done[i]) act.push_back(i);
    if (act.empty()) break;
    std::vector<int> act_c, act_r;
    for (int i : act) (coarse[i] ? act_c : act_r).push_back(i);
    // ---- filter: Q = sum_j w_j (z_j - B)^{-1} Y (+ conj(w_j)(z_j - B)^{-H} Y)
    {
      std::vector<c128*> Yc(nslice), Qc(nslice);
      std::vector<int64_t> lds(nslice, n);
      for (int i = 0; i < nslice; ++i) {
        Yc[i] = sb[i].Y;
        Qc[i] = sb[i].Q;
        Xp[(size_t)i * P] = sb[i].X;  // X and Y trade places every iteration
      }
      if (!act_c.empty())
        FB_TRY(filter_apply<R>(bd, f, ne, act_c, m0, Yc.data(), lds.data(), Qc.data(),
                               lds.data(), Xp.data(), P, acc_dev, zsys, wsys, cplx,
                               o->batched != 0, false, o->ir_tol, o->ir_max, false, rb, sys_res,
                               sys_pass, nullptr, st, nullptr));
      if (!act_r.empty())
        FB_TRY(filter_apply<R>(bd, f, ne, act_r, m0, Yc.data(), lds.data(), Qc.data(),
                               lds.data(), Xp.data(), P, acc_dev, zsys, wsys, cplx,
                               o->batched != 0, ir, o->ir_tol, o->ir_max, ir, rb, sys_res,
                               sys_pass, nullptr, st, ir ? &fbuf.fb : nullptr));
      for (int i : act)
        for (int j = 0; j < ne; ++j)
          if (sys_pass[i * ne + j] < 0) fellback[i] = 1;
    }
    std::vector<int> path(nslice, 0);
    FB_TRY(ortho_rr<R>(bd, nslice, act, m0, kept, path, fbuf, st));
    for (int i : act) {
      int m = m0[i], k = kept[i];
      if (k <= 0) continue;
      // X becomes the next start block
      if (k < m)  // rank-deficient filter output: keep the trailing start vectors
        FB_HIP(hipMemcpy2DAsync(sb[i].X + (size_t)k * n, n * sizeof(c128), sb[i].Y + (size_t)k * n,
                                n * sizeof(c128), n * sizeof(c128), m - k,
                                hipMemcpyDeviceToDevice, st));
      hl[i].resize(k);
      hr[i].resize(k);
      FB_HIP(hipMemcpyAsync(hl[i].data(), sb[i].lam, sizeof(double) * k, hipMemcpyDeviceToHost, st));
      FB_HIP(hipMemcpyAsync(hr[i].data(), sb[i].res, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    }
    FB_HIP(hipStreamSynchronize(st));
    for (int i : act) {
      std::swap(sb[i].Y, sb[i].X);  // next start block = all Ritz vectors
      iters[i] = it;
      int k = kept[i], g = 0, in = 0;
      for (int c = 0; c < k; ++c) {
        bool ins = hl[i][c] >= lo[i] && hl[i][c] < hi[i];
        in += ins;
        g += ins && hr[i][c] <= o->tol;
      }
      good[i] = g;
      inside[i] = in;
      if (g == mexp[i]) done[i] = 1;
      if (coarse[i] && !done[i]) {
        // refinement from here on once the m-th smallest in-slice residual
        // is at ir_from
        std::vector<double> rin;
        for (int c = 0; c < k; ++c)
          if (hl[i][c] >= lo[i] && hl[i][c] < hi[i]) rin.push_back(hr[i][c]);
        std::sort(rin.begin(), rin.end());
        const int need = std::max(mexp[i], 1);
        const bool near = (int)rin.size() >= need && rin[need - 1] <= o->ir_from;
        if (near || ++ncoarse[i] >= kCoarseIters) coarse[i] = 0;
      }
    }
  }

  // ---- outputs: converged in-slice pairs first (ascending), then the rest
  int nbad = 0;
  for (int i = 0; i < nslice; ++i) {
    if (info[i] == 5) {
      ++nbad;
      continue;
    }
    int m = m0[i], k = kept[i];
    std::vector<int32_t> perm;
    std::vector<double> ev, rs;
    for (int c = 0; c < k; ++c)
      if (hl[i][c] >= lo[i] && hl[i][c] < hi[i] && hr[i][c] <= o->tol) perm.push_back(c);
    for (int c = 0; c < k; ++c)
      if (!(hl[i][c] >= lo[i] && hl[i][c] < hi[i] && hr[i][c] <= o->tol)) perm.push_back(c);
    for (int c = k; c < m; ++c) perm.push_back(c);
    for (int c = 0; c < m; ++c) {
      int p = perm[c];
      ev.push_back(p < k ? hl[i][p] : NAN);
      rs.push_back(p < k ? hr[i][p] : INFINITY);
    }
    m_found[i] = good[i];
    if (done[i])
      info[i] = fellback[i] ? 3 : (k < m) ? 4 : 0;
    else
      info[i] = (good[i] > mexp[i] || inside[i] < mexp[i]) ? 2 : 1;
    if (info[i] == 1 || info[i] == 2) ++nbad;
    FB_HIP(hipMemcpyAsync(perm_dev, perm.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    FB_TRY(store_cols(sb[i].Y, n, Y[i], ldy[i], !cplx, n, m, perm_dev, st));
    FB_HIP(hipMemcpyAsync(evals[i], ev.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    FB_HIP(hipMemcpyAsync(resid[i], rs.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    FB_HIP(hipStreamSynchronize(st));
  }
  return nbad;
}

// Slices are processed in waves: as many slices per wave (all of them if
// they fit) and as many (node, direction) pairs per batched launch as the
// HBM budget allows, choosing the pair that gives the most solve jobs per
// launch.
template <typename R>
int feast_impl(const fb_band* B, int nslice, const double* lo, const double* hi, const int32_t* m0,
               const int32_t* m_expected, void* const* Y, const int64_t* ldy,
               double* const* evals, double* const* resid, int32_t* m_found, int32_t* iters,
               int32_t* info, const fb_feast_opts* o, void* work, size_t* lwork, hipStream_t st) {
  const bool ir = o->precision == 1;
  const int ne = o->n_nodes;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  double* fpart = ar.take<double>((size_t)kFiniteParts * std::max(nslice, 1));
  const int64_t n = B->n;
  const bool cplx = B->dtype == FB_COMPLEX128;
  int maxm = 1;
  for (int i = 0; i < nslice; ++i) maxm = std::max(maxm, (int)m0[i]);
  const int npair = ne * (cplx ? 2 : 1);
  double budget = o->hbm_budget;
  if (!(budget > 0)) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
    budget = 0.5 * (double)tot;
  }
  const size_t used0 = ar.used;
  int W = 1, P = 1;
  {
    long best = -1;
    for (int w = nslice; w >= 1; --w) {
      Arena q;
      q.used = used0;
      FeastBufs<R> tmp;
      carve_feast<R>(q, bd, w, maxm, ne, ir, 1, tmp);
      const size_t per_pair = (size_t)w * n * maxm * sizeof(c128);
      if ((double)q.used > budget && w > 1) continue;
      const int p = pairs_per_launch(budget, o->pairs, o->batched != 0, npair,
                                     q.used - per_pair * 0, per_pair);
      const long score = (long)w * p;
      if (score > best) {
        best = score;
        W = w;
        P = p;
      }
      if (w == nslice && (p == npair || o->batched == 0)) break;  // everything in one wave
    }
  }
  FeastBufs<R> fbuf;
  carve_feast<R>(ar, bd, W, maxm, ne, ir, P, fbuf);
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  FB_TRY(check_finite_blocks(nslice, Y, ldy, m0, n, cplx, fpart, st));
  int nbad = 0;
  for (int w0 = 0; w0 < nslice; w0 += W) {
    const int nw = std::min(W, nslice - w0);
    int rc = feast_wave<R>(bd, nw, lo + w0, hi + w0, m0 + w0,
                           m_expected ? m_expected + w0 : nullptr, Y + w0, ldy + w0, evals + w0,
                           resid + w0, m_found + w0, iters + w0, info + w0, o, fbuf, st);
    if (rc < 0) return rc;
    nbad += rc;
  }
  return nbad;
}

}  // namespace fb

using namespace fb;

extern "C" int feast_band_slice(const fb_band* B, int32_t nslice, const double* lo,
                                const double* hi, const int32_t* m0, const int32_t* m_expected,
                                void* const* Y, const int64_t* ldy, double* const* evals,
                                double* const* resid, int32_t* m_found, int32_t* iters,
                                int32_t* info, const fb_feast_opts* o, void* work,
                                size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (nslice < 0) return -2;
  if (nslice > 0 && (!lo || !hi)) return -3;
  if (nslice > 0 && !m0) return -5;
  if (nslice > 0 && (!Y || !ldy)) return -7;
  if (nslice > 0 && (!evals || !resid)) return -9;
  if (nslice > 0 && (!m_found || !iters || !info)) return -11;
  if (!o) return -14;
  if (!lwork) return -16;
  if (o->n_nodes < 1 || o->n_nodes > 64 || !(o->tol > 0) || o->max_iter < 1) return -14;
  if (!contour_ok(o->rule, o->ratio)) return -14;
  if (o->precision != 0 && o->precision != 1) return -14;
  if (o->precision == 1 && (!(o->ir_tol > 0) || o->ir_max < 0)) return -14;
  if (o->graph != 0 && o->graph != 1) return -14;
  if (!tune_cache_ok(o->tune_cache)) return -14;
  for (int i = 0; i < nslice; ++i) {
    if (!isfinite(lo[i]) || !isfinite(hi[i]) || !(lo[i] < hi[i])) return -3;
    if (m0[i] < 1 || m0[i] > 4096 || m0[i] > B->n) return -5;
    if (m_expected && m_expected[i] < 0) return -6;
    if (!Y[i] || ldy[i] < B->n) return -7;
    if (!evals[i] || !resid[i]) return -9;
  }
  if (nslice == 0) {
    if (!work) *lwork = 0;
    return 0;
  }
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == 1)
    return feast_impl<float>(B, nslice, lo, hi, m0, m_expected, Y, ldy, evals, resid, m_found,
                             iters, info, o, work, lwork, st);
  return feast_impl<double>(B, nslice, lo, hi, m0, m_expected, Y, ldy, evals, resid, m_found,
                            iters, info, o, work, lwork, st);
}

namespace fb {

template <typename R>
int filter_impl(const fb_band* B, int nslice, const double* lo, const double* hi, const int32_t* m,
                const void* const* Y, const int64_t* ldy, void* const* Q, const int64_t* ldq,
                double* resid, int32_t* passes, const fb_feast_opts* o, void* work,
                size_t* lwork, hipStream_t st) {
  const bool ir = o->precision == 1;
  const bool need_res = ir || resid != nullptr;
  const int ne = o->n_nodes;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  double* fpart = ar.take<double>((size_t)kFiniteParts * std::max(nslice, 1));
  const int64_t n = B->n;
  const bool cplx = B->dtype == FB_COMPLEX128;
  const int nsys = nslice * ne;
  FactorBufs<R> f;
  carve_factors<R>(ar, bd, nsys, f);
  FactorBufs<double> f64fb;
  C128Fallback fbk;
  if (ir) {
    fbk.cap = fallback_cap(nsys);
    carve_factors<double>(ar, bd, fbk.cap, f64fb);
    fbk.f = &f64fb;
  }
  std::vector<c128*> Yc(nslice), Qc(nslice);
  std::vector<int64_t> ldyc(nslice), ldqc(nslice);
  for (int i = 0; i < nslice; ++i) {
    if (cplx) {
      Yc[i] = (c128*)Y[i];
      Qc[i] = (c128*)Q[i];
      ldyc[i] = ldy[i];
      ldqc[i] = ldq[i];
    } else {  // real B: complex working copies of Y and Q
      Yc[i] = ar.take<c128>((size_t)n * std::max(m[i], 1));
      Qc[i] = ar.take<c128>((size_t)n * std::max(m[i], 1));
      ldyc[i] = ldqc[i] = n;
    }
  }
  AccJob* acc_dev = ar.take<AccJob>(nslice);
  const int tile = solve_tile<R>(bd.b);
  int max_jobs = 0;
  size_t cols = 0;
  for (int i = 0; i < nslice; ++i) {
    max_jobs += (m[i] + tile - 1) / tile;
    cols += std::max(m[i], 1);
  }
  const int npair = ne * (cplx ? 2 : 1);
  const int P = pairs_per_launch(o->hbm_budget, o->pairs, o->batched != 0, npair,
                                 ar.used + refine_bytes(bd, tile, max_jobs, ir, need_res),
                                 (size_t)n * cols * sizeof(c128));
  std::vector<c128*> Xp((size_t)nslice * P);
  for (int i = 0; i < nslice; ++i)
    for (int p = 0; p < P; ++p) Xp[(size_t)i * P + p] = ar.take<c128>((size_t)n * std::max(m[i], 1));
  RefineBufs rb;
  carve_refine(ar, bd, tile, max_jobs * P, ir, need_res, rb);
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  FB_TRY(check_finite_blocks(nslice, Y, ldy, m, n, cplx, fpart, st));
  std::vector<c128> zsys(nsys), wsys(nsys);
  std::vector<double> zh(2 * nsys);
  for (int i = 0; i < nslice; ++i) {
    std::vector<c128> z, w;
    contour(lo[i], hi[i], ne, o->rule, o->ratio, z, w);
    for (int j = 0; j < ne; ++j) {
      zsys[i * ne + j] = z[j];
      wsys[i * ne + j] = w[j];
      zh[2 * (i * ne + j)] = z[j].x;
      zh[2 * (i * ne + j) + 1] = z[j].y;
    }
  }
  std::vector<int> act;
  for (int i = 0; i < nslice; ++i)
    if (m[i] > 0) act.push_back(i);
  std::vector<double> sys_res(nsys, 0.0);
  std::vector<int32_t> sys_pass(nsys, 0);
  int unconverged = 0;
  const int npair_all = ne * (cplx ? 2 : 1);
  bool done = false;
  if (o->graph && st != nullptr && o->batched && P >= npair_all && npair_all <= kMaxPairs) {
    // graph form: the whole sweep (factorisations, solves, refinement passes,
    // node sum) is captured once per argument set and replayed; the tables
    // it reads are uploaded before every replay
    FB_HIP(hipMemcpyAsync(f.z, zh.data(), sizeof(c128) * nsys, hipMemcpyHostToDevice, st));
    const std::vector<std::pair<int, int>> pairs = node_pairs(ne, cplx);
    std::vector<SolveJob> jobs;
    std::vector<AccJob> aj;
    int maxm = 0;
    build_pair_jobs<R>(n, rb.tile, ne, act, m, Yc.data(), ldyc.data(), Qc.data(), ldqc.data(),
                       Xp.data(), P, pairs, 0, npair_all, -1, wsys, cplx, jobs, aj, maxm);
    RefinePlan plan;
    FB_TRY(refine_prepare<R>(bd, jobs, zsys, ir, o->ir_tol, o->ir_max, need_res, rb, plan, st));
    if (!aj.empty())
      FB_HIP(hipMemcpyAsync(acc_dev, aj.data(), sizeof(AccJob) * aj.size(), hipMemcpyHostToDevice, st));
    char key[512];
    snprintf(key, sizeof key, "%d|%p|%lld|%d|%d|%lld|%d|%d|%d|%d|%.17g|%d|%d|%p|%zu|%p",
             (int)sizeof(R), B->ab, (long long)n, B->b, B->dtype, (long long)B->ldab, nslice, ne,
             o->precision, o->ir_max, o->ir_tol, P, (int)need_res, work, *lwork, (void*)st);
    std::string k(key);
    for (int i = 0; i < nslice; ++i) {
      snprintf(key, sizeof key, "|%d:%p:%lld:%p:%lld", m[i], Y[i], (long long)ldy[i], Q[i],
               (long long)ldq[i]);
      k += key;
    }
    hipError_t le = hipSuccess;
    if (!graph_launch(k, st, &le)) {
      hipGraphExec_t exec = nullptr;
      FB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      int rc = launch_lu_impl<R>(bd, nsys, f.z, f.mats, f.matsT, f.perm, f.info, f.scratch,
                                 f.lscr, st);
      for (size_t a = 0; rc == 0 && !cplx && a < act.size(); ++a) {
        const int i = act[a];
        rc = gather_cols(Y[i], ldy[i], true, Yc[i], n, n, m[i], nullptr, nullptr, st);
      }
      if (rc == 0) rc = refine_launch<R>(bd, f.mats, f.matsT, f.perm, plan, rb, st);
      if (rc == 0) rc = accumulate_pairs(acc_dev, (int)aj.size(), n, maxm, st);
      for (size_t a = 0; rc == 0 && !cplx && a < act.size(); ++a) {
        const int i = act[a];
        rc = store_cols(Qc[i], n, Q[i], ldq[i], true, n, m[i], nullptr, st);
      }
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (rc == 0 && ec != hipSuccess) rc = -1000 - (int)ec;
      if (rc == 0) {
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) rc = -1000 - (int)ei;
      }
      if (g) (void)hipGraphDestroy(g);
      if (rc != 0) return rc;
      le = graph_store_launch(k, exec, st);
    }
    FB_HIP(le);
    FB_TRY(factor_check<R>(nsys, f, st));
    int stagnated = 0;
    FB_TRY(refine_finish<R>(bd, jobs, zsys, plan, rb, sys_res, sys_pass, &unconverged, st, nullptr,
                            &stagnated));
    if (stagnated == 0) {
      done = true;
    } else {  // a refinement stagnated: the direct sweep redoes it with the fallback
      std::fill(sys_res.begin(), sys_res.end(), 0.0);
      std::fill(sys_pass.begin(), sys_pass.end(), 0);
      unconverged = 0;
    }
  }
  if (!done) {
    FB_TRY(factor_systems<R>(bd, nsys, zh.data(), f, st));
    for (int i : act)
      if (!cplx) FB_TRY(gather_cols(Y[i], ldy[i], true, Yc[i], n, n, m[i], nullptr, nullptr, st));
    FB_TRY(filter_apply<R>(bd, f, ne, act, m, Yc.data(), ldyc.data(), Qc.data(), ldqc.data(),
                           Xp.data(), P, acc_dev, zsys, wsys, cplx, o->batched != 0, ir, o->ir_tol,
                           o->ir_max, need_res, rb, sys_res, sys_pass, &unconverged, st,
                           ir ? &fbk : nullptr));
    if (!cplx)
      for (int i : act) FB_TRY(store_cols(Qc[i], n, Q[i], ldq[i], true, n, m[i], nullptr, st));
  }
  FB_HIP(hipStreamSynchronize(st));
  int nbad = 0;
  for (int i = 0; i < nslice; ++i) {
    double r = 0.0;
    int p = 0;
    bool fell = false;  // a system re-solved in complex128
    for (int j = 0; j < ne; ++j) {
      r = std::max(r, sys_res[i * ne + j]);
      p = std::max(p, sys_pass[i * ne + j]);
      fell = fell || sys_pass[i * ne + j] < 0;
    }
    if (resid) resid[i] = r;
    if (passes) passes[i] = fell ? -1 : p;
    if (ir && !(r <= o->ir_tol) && m[i] > 0) ++nbad;
  }
  return nbad;
}

}  // namespace fb

extern "C" int feast_filter(const fb_band* B, int32_t nslice, const double* lo, const double* hi,
                            const int32_t* m, const void* const* Y, const int64_t* ldy,
                            void* const* Q, const int64_t* ldq, double* resid, int32_t* passes,
                            const fb_feast_opts* o, void* work, size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (nslice < 0) return -2;
  if (nslice > 0 && (!lo || !hi)) return -3;
  if (nslice > 0 && !m) return -5;
  if (nslice > 0 && (!Y || !ldy)) return -6;
  if (nslice > 0 && (!Q || !ldq)) return -8;
  if (!o) return -12;
  if (!lwork) return -14;
  if (o->n_nodes < 1 || o->n_nodes > 64) return -12;
  if (!contour_ok(o->rule, o->ratio)) return -12;
  if (o->precision != 0 && o->precision != 1) return -12;
  if (o->precision == 1 && (!(o->ir_tol > 0) || o->ir_max < 0)) return -12;
  if (o->graph != 0 && o->graph != 1) return -12;
  if (!tune_cache_ok(o->tune_cache)) return -12;
  for (int i = 0; i < nslice; ++i) {
    if (!isfinite(lo[i]) || !isfinite(hi[i]) || !(lo[i] < hi[i])) return -3;
    if (m[i] < 0) return -5;
    if (m[i] > 0 && (!Y[i] || ldy[i] < B->n)) return -6;
    if (m[i] > 0 && (!Q[i] || ldq[i] < B->n)) return -8;
  }
  if (nslice == 0) {
    if (!work) *lwork = 0;
    return 0;
  }
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == 1)
    return filter_impl<float>(B, nslice, lo, hi, m, Y, ldy, Q, ldq, resid, passes, o, work, lwork,
                              st);
  return filter_impl<double>(B, nslice, lo, hi, m, Y, ldy, Q, ldq, resid, passes, o, work, lwork,
                             st);
}

extern "C" int fb_contour(double lo, double hi, int32_t k, int32_t rule, double ratio, double* z,
                          double* w) {
  if (!isfinite(lo)) return -1;
  if (!isfinite(hi) || !(hi > lo)) return -2;
  if (k < 1 || k > 64) return -3;
  if (rule < 0 || rule > 2) return -4;
  if (!contour_ok(rule, ratio)) return -5;
  if (!z) return -6;
  if (!w) return -7;
  std::vector<c128> zz, ww;
  contour(lo, hi, k, rule, ratio, zz, ww);
  for (int j = 0; j < k; ++j) {
    z[2 * j] = zz[j].x;
    z[2 * j + 1] = zz[j].y;
    w[2 * j] = ww[j].x;
    w[2 * j + 1] = ww[j].y;
  }
  return 0;
}

extern "C" int band_rayleigh_ritz(const fb_band* B, int32_t nblk, const int32_t* m,
                                  const void* const* Q, const int64_t* ldq, void* const* X,
                                  const int64_t* ldx, double* const* evals, double* const* resid,
                                  int32_t* rank, int32_t* path, void* work, size_t* lwork,
                                  void* stream) {
  if (check_band(B)) return -1;
  if (nblk < 0) return -2;
  if (nblk > 0 && !m) return -3;
  if (nblk > 0 && (!Q || !ldq)) return -4;
  if (nblk > 0 && (!X || !ldx)) return -6;
  if (nblk > 0 && (!evals || !resid)) return -8;
  if (nblk > 0 && !rank) return -10;
  if (!lwork) return -13;
  int maxm = 1;
  for (int i = 0; i < nblk; ++i) {
    if (m[i] < 0 || m[i] > 4096 || m[i] > B->n) return -3;
    if (m[i] > 0 && (!Q[i] || ldq[i] < B->n)) return -4;
    if (m[i] > 0 && (!X[i] || ldx[i] < B->n)) return -6;
    if (m[i] > 0 && (!evals[i] || !resid[i])) return -8;
    maxm = std::max(maxm, (int)m[i]);
  }
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st, false));
  FeastBufs<double> fbuf;
  carve_feast<double>(ar, bd, std::max(nblk, 1), maxm, 0, false, 1, fbuf);
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  const int64_t n = bd.n;
  const bool cplx = bd.cplx;
  std::vector<int> act, kept(nblk, 0), pth(nblk, 0);
  for (int i = 0; i < nblk; ++i) {
    if (m[i] <= 0) continue;
    act.push_back(i);
    FB_TRY(gather_cols(Q[i], ldq[i], !cplx, fbuf.sb[i].Q, n, n, m[i], nullptr, nullptr, st));
  }
  FB_TRY(ortho_rr<double>(bd, nblk, act, m, kept, pth, fbuf, st));
  for (int i : act) {
    const int k = kept[i];
    if (k <= 0) continue;
    FB_TRY(store_cols(fbuf.sb[i].X, n, X[i], ldx[i], !cplx, n, k, nullptr, st));
    FB_HIP(hipMemcpyAsync(evals[i], fbuf.sb[i].lam, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
    FB_HIP(hipMemcpyAsync(resid[i], fbuf.sb[i].res, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  }
  FB_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nblk; ++i) {
    rank[i] = kept[i];
    if (path) path[i] = pth[i];
  }
  return 0;
}
